"""Benchmark of the MI355X Maxwell-Bloch hot path.

Default workload: the three-level Lambda medium on 32768 cells for 200000
steps (16 seeded materials, Gaussian pulse-train drive, populations recorded
at 64 probes every 10 steps).  One benchmark "step" is one complete solve of
that workload (all 200000 time steps) with its inputs resident in device
memory; the initial state is restored from a device copy between solves.

Printed: one JSON line with cell-updates/s of the FP32 temporally blocked
path (``value``), the FP64 two-launch and blocked paths on the same
workload, their errors against the FP64 oracle on a bounded prefix (the same
oracle run is the CPU baseline), the roofline of the dominant kernel and,
unless disabled, the batched parameter sweep and a serving trace with
p50/p99 solve latency.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# the serving leg runs one stream per level count; give HIP enough hardware
# queues (read at HIP start-up) that they do not share one
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4) < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

import paper_2005_05412_amd as mb  # noqa: E402
import workloads as W  # noqa: E402
from workloads.errors import max_error  # noqa: E402

PEAK = {"fp32_tflops": 157.3, "fp64_tflops": 78.6, "hbm_gbs": 8000.0}


def flops_per_cell_update(n):
    """Algorithmic flops of one cell-update: Yee updates (8), field phases as
    complex multiplies on the N(N-1)/2 coherences (6 each), polarization
    readout (2M) and the affine propagator (2M^2 + M), M = N^2 - 1."""
    m = n * n - 1
    return 8 + 6 * (n * (n - 1) // 2) + 2 * m + 2 * m * m + m


def flops_issued_per_cell_update(n):
    """Flops the kernels issue per cell-update: the state is kept in the basis of the
    operators, so the field part goes through the eigenbasis coherences, z = t0 + T x
    (2KM), their increments (6 per pair), p = p0 + at.x + as.d (2(M+K)) and
    x += bf + (A - I) x + (A S) d (2M(M+K) + 2M), K = N(N-1), besides the Yee updates (8)."""
    m, k = n * n - 1, n * (n - 1)
    return 8 + 2 * k * m + 6 * (k // 2) + 2 * (m + k) + 2 * m * (m + k) + 2 * m


def alu_tflops(n, cell_updates, ms):
    """Algorithmic TFLOP/s of cell_updates N-level cell-updates in ms milliseconds."""
    return flops_per_cell_update(n) * cell_updates / (ms * 1e-3) / 1e12


def bytes_per_cell_update(n, prec):
    """Algorithmic HBM bytes of one cell-update: read and write of E, H and the M density reals."""
    return 2 * (n * n + 1) * (8 if prec == 64 else 4)


KERNEL_SOURCES = ("paper_2005_05412_amd/csrc/kernels.hip", "paper_2005_05412_amd/csrc/engine.hpp")


def kernel_source_hash():
    """Short SHA-256 of the device sources; counter figures are tied to it."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


PERSIST_CHUNKS = 4096  # chunks one persistent launch of mb_run covers at most


def measured_traffic(kernel, workload, depth, steps):
    """HBM bytes per launch of `kernel` from a committed counter summary.

    The summaries under profiles/ carry lines of the form
    ``traffic-record: kernel=K workload=W depth=D steps=T source=S bytes_per_launch=B``
    (T: time steps one launch advances) where B is FETCH_SIZE + WRITE_SIZE per
    dispatch, each scaled by what the counter reads for a device copy of known
    size.  The figure is used only while the device sources still hash to S;
    otherwise None.
    """
    src = kernel_source_hash()
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    for name in sorted(os.listdir(pdir)):
        with open(os.path.join(pdir, name), encoding="utf-8", errors="replace") as f:
            for line in f:
                line = line.strip().strip("`")
                if not line.startswith("traffic-record:"):
                    continue
                kv = dict(t.split("=", 1) for t in line.split()[1:] if "=" in t)
                if (kv.get("kernel") == kernel and kv.get("workload") == workload
                        and kv.get("depth") == str(depth) and kv.get("steps") == str(steps)
                        and kv.get("source") == src):
                    return float(kv["bytes_per_launch"])
    return None


class Hip:
    """Minimal HIP runtime access (stream, events, synchronisation) via ctypes."""

    def __init__(self):
        self.lib = ctypes.CDLL("libamdhip64.so")

    def sync(self):
        rc = self.lib.hipDeviceSynchronize()
        if rc != 0:
            raise RuntimeError(f"hipDeviceSynchronize failed: {rc}")

    def stream(self):
        s = ctypes.c_void_p()
        if self.lib.hipStreamCreateWithFlags(ctypes.byref(s), 1) != 0:
            raise RuntimeError("hipStreamCreateWithFlags failed")
        return s.value

    def event(self):
        e = ctypes.c_void_p()
        if self.lib.hipEventCreate(ctypes.byref(e)) != 0:
            raise RuntimeError("hipEventCreate failed")
        return e

    def record(self, ev, stream):
        self.lib.hipEventRecord(ev, ctypes.c_void_p(stream))

    def elapsed_ms(self, a, b):
        self.lib.hipEventSynchronize(b)
        ms = ctypes.c_float()
        self.lib.hipEventElapsedTime(ctypes.byref(ms), a, b)
        return ms.value

    def copy_calibration(self, nbytes):
        """One device-to-device copy of nbytes (a plain copy kernel of known traffic)."""
        src, dst = ctypes.c_void_p(), ctypes.c_void_p()
        if self.lib.hipMalloc(ctypes.byref(src), ctypes.c_size_t(nbytes)) != 0 or \
                self.lib.hipMalloc(ctypes.byref(dst), ctypes.c_size_t(nbytes)) != 0:
            raise RuntimeError("hipMalloc failed")
        self.lib.hipMemset(src, 1, ctypes.c_size_t(nbytes))
        self.sync()
        if self.lib.hipMemcpy(dst, src, ctypes.c_size_t(nbytes), 3) != 0:   # device to device
            raise RuntimeError("hipMemcpy failed")
        self.sync()
        self.lib.hipFree(src)
        self.lib.hipFree(dst)


def rel_err(prob, got, ref):
    """Relative max-norm error over the recorded traces (compared on the common prefix)."""
    n = min(min(len(got[r["name"]]), len(ref[r["name"]])) for r in prob["records"])
    return max_error(prob, got, ref, n_samples=n)


def timed_solves(hip, stream, solver, steps, warmup, n_launch):
    for _ in range(warmup):
        solver.reset(stream).run(-1, stream)
    hip.sync()
    evs = [(hip.event(), hip.event()) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        solver.reset(stream)
        hip.record(a, stream)
        solver.run(-1, stream)
        hip.record(b, stream)
    hip.sync()
    wall = time.perf_counter() - t0
    dev_ms = [hip.elapsed_ms(a, b) for a, b in evs]
    return wall, dev_ms


def stored_lambda3_records(prob):
    """The oracle's records of the full Lambda workload (tests/golden/oracle_lambda3.npz,
    written by tests/golden/make_oracle_records.py; every stride-th sample), or None."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_lambda3.npz")
    if not os.path.exists(path) or prob["nx"] != 32768 or prob["n_steps"] != 200000:
        return None
    # the records are those of weak coupling and the exact field step
    if prob.get("coupling", "weak") != "weak" or prob.get("field_step", "exact") != "exact":
        return None
    d = np.load(path)
    stride = int(d["lambda3/stride"])
    return {r["name"]: d["lambda3/" + r["name"]] for r in prob["records"]}, stride


def sweep_sub_batch(hip, stream, sims, log):
    """The first members of the batched sweep as one batch in three forms, each timed
    (HIP events, median of 3 after a warm-up): FP64 plain (two launches per step), FP64
    temporally blocked, FP32 temporally blocked."""
    cells = sum(p["nx"] * p["n_steps"] for p in sims)
    out = {"sims": len(sims), "cell_updates": cells, "unit": "cell-updates/s"}
    for key, prec, variant in (("fp64_plain", 64, "plain"), ("fp64_blocked", 64, "auto"),
                               ("fp32_blocked", 32, "auto")):
        log(f"[bench] sweep sub-batch of {len(sims)}: {key}")
        probs = [dict(p, precision=prec) for p in sims]
        bt = mb.Batch(probs, precision=prec, variant=variant)
        bt.run(stream=stream, use_graph=True)
        hip.sync()
        ms = []
        for _ in range(3):
            bt.reset(stream)
            a, b = hip.event(), hip.event()
            hip.record(a, stream)
            bt.run(stream=stream, use_graph=True)
            hip.record(b, stream)
            ms.append(hip.elapsed_ms(a, b))
        bt.close()
        out[key] = cells / (float(np.median(ms)) * 1e-3)
    out["fp32_blocked_over_fp64_plain"] = out["fp32_blocked"] / out["fp64_plain"]
    return out


def _oracle_prefix(args):
    """Worker: the FP64 oracle on the first n_steps of a workload (one BLAS thread);
    returns (steps, seconds, records)."""
    name, n_steps, budget_s = args
    from threadpoolctl import threadpool_limits
    from oracle import Oracle

    prob = _cpu_workload(name)
    with threadpool_limits(limits=1):
        orc = Oracle(prob)
        step_rec = max(r["interval"] for r in prob["records"])
        t0 = time.perf_counter()
        n = 0
        while n < min(n_steps, prob["n_steps"]):
            for _ in range(step_rec):
                orc.step()
            n += step_rec
            if budget_s is not None and time.perf_counter() - t0 > budget_s:
                break
        el = time.perf_counter() - t0
    return n, el, {k: np.array(v) for k, v in orc.records.items()}


def _cpu_workload(name):
    if name == "lambda3":
        return W.lambda3(precision=32)
    if name == "sit":
        return W.sit_2lvl()
    raise ValueError(name)


def host_cores():
    """Host cores this process may use (the GPU machine's share is 16 cores per GPU)."""
    return max(1, min(len(os.sched_getaffinity(0)), 16))


def cpu_baselines(budget_s, log):
    """The FP64 oracle on the host, before the GPU is touched (worker processes are
    forked): the Lambda workload's prefix on one thread alone, then the same prefix as
    independent solves on every host core at once, then the SIT workload in full on one
    thread."""
    import multiprocessing as mp

    cores = host_cores()
    log(f"[bench] oracle on the host: lambda3 prefix on 1 thread, then on {cores} cores; sit in full")
    n1, t1, rec1 = _oracle_prefix(("lambda3", 10 ** 9, budget_s))
    with mp.get_context("fork").Pool(cores) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_prefix, [("lambda3", n1, None)] * cores)
        tall = time.perf_counter() - t0
    nx = W.lambda3(precision=32)["nx"]
    n_sit, t_sit, rec_sit = _oracle_prefix(("sit", 10 ** 9, None))
    sit = W.sit_2lvl()
    return {
        "value": cores * nx * n1 / tall, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
        "sample": (f"first {n1} of 200000 steps of the same workload (all {nx} cells), numpy FP64: "
                   f"{cores} independent solves at once, one BLAS thread each, wall {tall:.1f} s"),
        "value_1thread": nx * n1 / t1, "seconds_1thread": t1,
        "per_process_s": [float(r[1]) for r in res],
        "sit_full_run": {"value": sit["nx"] * n_sit / t_sit, "unit": "cell-updates/s", "cores": 1,
                         "steps": n_sit, "seconds": t_sit,
                         "sample": "the SIT workload in full (1500 cells x 20000 steps), one thread"},
    }, n1, rec1, rec_sit


def levels_of(prob):
    """Level count of a problem's quantum material (0 for vacuum)."""
    for m in prob["materials"]:
        q = m["qm"]
        if q is not None:
            return 2 if q["kind"] == "2lvl" else len(q["h0_diag"])
    return 0


def run_serving(n_requests, rate, log, first_n=0):
    """Poisson trace through the continuous-batching server; latency = arrival to records on
    the host (also p50/p99 over the first first_n requests, for the FIFO comparison)."""
    log(f"[bench] serving {n_requests} requests at {rate:g}/s")
    trace = W.serve_trace(n_requests=n_requests, rate=rate, precision=32)
    srv = mb.Server(hbm_budget=16 << 30, max_slots=512, precision=32, chunk_steps=256)
    tickets = [srv.submit(p, t) for t, p in trace]
    offered = sum(p["nx"] * p["n_steps"] for _, p in trace) / max(trace[-1][0], 1e-9)
    t0 = time.perf_counter()
    srv.start()
    # progress every 20 s while the trace drains (poll: tickets that became final)
    n_final, t_log = 0, t0
    while n_final < len(tickets) and time.perf_counter() - t0 < 600:
        time.sleep(0.05)
        n_final += len(srv.poll(4096))
        if time.perf_counter() - t_log >= 20:
            t_log = time.perf_counter()
            log(f"[bench] serving: {n_final} of {len(tickets)} requests final after {t_log - t0:.0f} s")
    srv.drain(timeout_s=max(1.0, 600 - (time.perf_counter() - t0)))
    tw = time.perf_counter() - t0
    lat = []
    by_levels = {}
    for t, (_, p) in zip(tickets, trace):
        st, ta, tadm, td = srv.status(t)
        if st == 2:
            lat.append(td - ta)
            by_levels.setdefault(levels_of(p), []).append(td - ta)
    cu, busy, chunks = srv.stats()
    srv.close()
    lat = np.array(lat)
    if first_n:
        sub = lat[:first_n]
        first = {"requests": int(len(sub)), "p50_latency_s": float(np.percentile(sub, 50)),
                 "p99_latency_s": float(np.percentile(sub, 99))}
    return {"requests": len(trace), "done": int(len(lat)), "arrival_rate_per_s": rate,
            **({"first_requests": first} if first_n else {}),
            "offered_cell_updates_per_s": offered,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "p50_latency_s_by_levels": {str(k): float(np.percentile(v, 50)) for k, v in sorted(by_levels.items())},
            "value": cu / tw, "unit": "cell-updates/s", "wall_s": tw, "busy_s": busy, "chunks": int(chunks)}


def solve_median(hip, stream, prob, precision, variant="auto", reps=5):
    """Setup, one untimed (graph-capturing) run, then `reps` runs from the restored
    initial state timed with HIP events on the stream; the median device time (ms),
    the records of the last run and the tile shape."""
    s = mb.Solver(prob, precision=precision, variant=variant)
    s.run(-1, stream)
    hip.sync()
    ms = []
    for _ in range(reps):
        s.reset(stream)
        a, b = hip.event(), hip.event()
        hip.record(a, stream)
        s.run(-1, stream)
        hip.record(b, stream)
        ms.append(hip.elapsed_ms(a, b))
    hip.sync()
    rec = s.records()
    shape = s.shape()
    s.close()
    return float(np.median(ms)), rec, shape


def with_steps(prob, n_steps):
    p = dict(prob)
    p["n_steps"] = int(n_steps)
    return p


def crossing_step(prob, got, ref, tol):
    """First recorded step at which the per-trace error of got against ref, taken over
    the samples up to it, exceeds tol (None if it never does)."""
    from workloads.errors import floor_of
    first = None
    for r in prob["records"]:
        a, b = np.asarray(got[r["name"]]), np.asarray(ref[r["name"]])
        n = min(len(a), len(b))
        if n == 0:
            continue
        err = np.maximum.accumulate(np.abs(a[:n] - b[:n]))
        scale = np.maximum(np.maximum.accumulate(np.abs(b[:n])), floor_of(prob, r["quantity"]))
        bad = np.nonzero(err / scale > tol)[0]
        if len(bad):
            step = int((bad[0] + 1) * r["interval"])
            first = step if first is None else min(first, step)
    return first


def leg(hip, stream, name, prob, log, timing_steps=None, error_steps=None, ref=None):
    """FP32 and FP64 throughput of one workload (median of 5 event-timed solves of
    timing_steps steps, default all), and the FP32 error against FP64 over error_steps
    (default all) with the step at which it first exceeds 1e-4; ref: oracle records of
    the workload (then the errors of both precisions against them as well)."""
    tp = with_steps(prob, timing_steps) if timing_steps else prob
    log(f"[bench] {name}: {tp['nx']} cells, {tp['n_steps']} steps, median of 5, fp32 / fp64")
    ms32, r32, sh32 = solve_median(hip, stream, tp, 32)
    ms64, r64, sh64 = solve_median(hip, stream, tp, 64)
    cells = tp["nx"] * tp["n_steps"]
    n = levels_of(prob)
    out = {"nx": prob["nx"], "n_steps_timed": tp["n_steps"], "unit": "cell-updates/s",
           "fp32": cells / (ms32 * 1e-3), "fp64": cells / (ms64 * 1e-3),
           "fp32_ms_median": ms32, "fp64_ms_median": ms64,
           "fp32_tflops_algorithmic": alu_tflops(n, cells, ms32) if n else None,
           "shape_fp32": list(sh32), "shape_fp64": list(sh64)}
    if error_steps != timing_steps:
        ep = with_steps(prob, error_steps) if error_steps else prob
        log(f"[bench] {name}: {ep['n_steps']}-step runs for the FP32 error")
        _, r32, _ = solve_median(hip, stream, ep, 32, reps=1)
        _, r64, _ = solve_median(hip, stream, ep, 64, reps=1)
    else:
        ep = tp
    out["n_steps_error"] = ep["n_steps"]
    out["fp32_vs_fp64_max_rel_err"] = max_error(ep, r32, r64)
    out["fp32_vs_fp64_crosses_1e-4_at_step"] = crossing_step(ep, r32, r64, 1e-4)
    if ref is not None:
        out["fp32_vs_oracle_max_rel_err"] = rel_err(ep, r32, ref)
        out["fp64_vs_oracle_max_rel_err"] = rel_err(ep, r64, ref)
    return out


def other_configs(hip, stream, log, sit_ref=None):
    """Throughput (median of 5 event-timed solves) and FP32 error of the other scenario shapes."""
    res = {}
    res["sit_2lvl"] = leg(hip, stream, "sit 2-level", W.sit_2lvl(), log, ref=sit_ref)
    # 1e6 steps: timed on 50000, FP32 against FP64 over 200000
    res["qcl_6lvl"] = leg(hip, stream, "qcl-like 6-level", W.qcl6(), log, timing_steps=50000, error_steps=200000)
    res["qcl_5lvl_comb"] = leg(hip, stream, "paper's 5-level comb (R = 0.8)", W.qcl5_comb(), log,
                               timing_steps=50000, error_steps=200000)
    p = W.lambda3()
    p["coupling"] = "strong"
    res["lambda3_strong_coupling"] = leg(hip, stream, "lambda3 strong coupling", p, log)
    p = W.lambda3()
    p["field_step"] = "cayley"
    res["lambda3_cayley_field_step"] = leg(hip, stream, "lambda3 Cayley field step", p, log)
    scal = {}
    for n in range(2, 9):
        r = leg(hip, stream, f"anharmonic ladder N={n}", W.ladder(n), log)
        r["flop_per_cell_update"] = flops_per_cell_update(n)
        scal[str(n)] = r
    res["ladder_n_scaling"] = {"nx": 8192, "n_steps": 20000, "unit": "cell-updates/s", "by_levels": scal}
    log("[bench] sweep x8: 2048 sims fp32 (state beyond the 256 MB last-level cache)")
    sims = W.sweep(n_sims=2048, precision=32, seed=W.SEED_BASE + 13)
    bcells = sum(q["nx"] * q["n_steps"] for q in sims)
    bt = mb.Batch(sims, precision=32, variant="auto")
    x8mode = bt.run_mode()
    bt.run(stream=stream, use_graph=True)
    hip.sync()
    bt.reset(stream)
    hip.sync()
    t0 = time.perf_counter()
    bt.run(stream=stream, use_graph=True)
    hip.sync()
    tb = time.perf_counter() - t0
    beff = sum(bytes_per_cell_update(2 if k % 2 == 0 else 3, 32) * q["nx"] * q["n_steps"]
               for k, q in enumerate(sims)) / tb / 1e9
    # E, H and the density entries with their FP32 compensation (3 and 8 entries)
    state_bytes = sum(q["nx"] * (2 + 2 * (3 if k % 2 == 0 else 8)) * 4 for k, q in enumerate(sims))
    res["sweep_x8"] = {"sims": len(sims), "cell_updates": bcells, "value": bcells / tb, "unit": "cell-updates/s",
                       "launch_form": x8mode,
                       "wall_s": tb, "state_bytes_one_buffer": state_bytes,
                       "bytes_algorithmic_per_s": beff * 1e9, "shape": list(bt.shape())}
    bt.close()
    return res


def plain_fifo(trace, log):
    """The baseline server: requests one after another in arrival order, each solved by
    the plain FP64 kernel (two launches per step); latency = arrival to records on the
    host, arrivals replayed on the wall clock."""
    log(f"[bench] FIFO plain FP64 serving of {len(trace)} requests")
    lat, by_levels = [], {}
    cu = 0
    t0 = time.perf_counter()
    for ta, p in trace:
        now = time.perf_counter() - t0
        if now < ta:
            time.sleep(ta - now)
        s = mb.Solver(p, precision=64, variant="plain")
        s.run()
        s.records()
        s.close()
        done = time.perf_counter() - t0
        lat.append(done - ta)
        by_levels.setdefault(levels_of(p), []).append(done - ta)
        cu += p["nx"] * p["n_steps"]
        if len(lat) % 10 == 0:
            log(f"[bench] FIFO: {len(lat)} of {len(trace)} requests done after {done:.0f} s")
    tw = time.perf_counter() - t0
    lat = np.array(lat)
    return {"requests": len(trace), "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "p50_latency_s_by_levels": {str(k): float(np.percentile(v, 50)) for k, v in sorted(by_levels.items())},
            "value": cu / tw, "unit": "cell-updates/s", "wall_s": tw}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nx", type=int, default=32768)
    ap.add_argument("--nt", type=int, default=200000)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--depth", type=int, default=0)
    ap.add_argument("--lanes", type=int, default=0, help="waves per 64 cells (1, 2, 4, 8; 0 = tuned)")
    ap.add_argument("--regs", action="store_true", help="with --block/--depth/--lanes: coefficients in registers")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-sub32", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--only", default="",
                    help="comma list of optional legs to run (fp64,cpu,batch,sub32,configs,serve); others are skipped")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests of the 200/s Poisson trace (2000 = the full 10 s trace)")
    ap.add_argument("--coupling", default="weak", choices=("weak", "strong"),
                    help="coupling of the main workload's density step to E (weak: rho half a step after E)")
    ap.add_argument("--field-step", default="exact", choices=("exact", "cayley"),
                    help="field part of the density step of the main workload (exact exponential or Cayley)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run one device-to-device copy of this size (counter calibration)")
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    if args.only:
        keep = set(args.only.split(","))
        for leg in ("fp64", "cpu", "batch", "sub32", "configs", "serve"):
            if leg not in keep:
                setattr(args, "no_" + leg, True)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        return 2
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    # ---- CPU baseline first: its worker processes are forked before the GPU is touched
    cpu = None
    if not args.no_cpu:
        cpu, n_cpu, ref_prefix, ref_sit = cpu_baselines(args.cpu_seconds, log)
    hip = Hip()
    stream = hip.stream()
    if args.copy_bytes > 0:
        hip.copy_calibration(args.copy_bytes)
    prob = W.lambda3(nx=args.nx, n_steps=args.nt, precision=32)
    prob["field_step"] = args.field_step
    prob["coupling"] = args.coupling
    wname = "lambda3-3lvl" + ("-cayley" if args.field_step == "cayley" else "") + \
        ("-strong" if args.coupling == "strong" else "")
    n_levels = 3
    cells = prob["nx"] * prob["n_steps"]

    # ---- main leg: FP32 temporally blocked -------------------------------------------
    log(f"[bench] lambda3 fp32 blocked nx={prob['nx']} nt={prob['n_steps']}")
    variant = ("blocked_regs" if args.regs else "blocked") if (args.block or args.depth or args.lanes) else "auto"
    t_setup = time.perf_counter()
    s32 = mb.Solver(prob, precision=32, variant=variant, block=args.block, depth=args.depth, lanes=args.lanes)
    t_setup = time.perf_counter() - t_setup
    block, depth, regs, lanes = s32.shape()
    log(f"[bench] tile shape block={block} depth={depth} regs={regs} lanes={lanes} "
        f"(setup incl. tuning {t_setup:.2f} s)")
    # full chunks of `depth` steps run as persistent launches (up to
    # PERSIST_CHUNKS chunks each) when the tiles fit on the device at once,
    # else one launch per chunk; the tail chunk is a launch of its own
    persistent = s32.persistent()
    n_chunks = math.ceil(prob["n_steps"] / depth)
    full, tail = divmod(prob["n_steps"], depth)
    n_launch = (math.ceil(full / PERSIST_CHUNKS) + (1 if tail else 0)) if persistent else n_chunks
    steps_per_launch = prob["n_steps"] // n_launch
    wall, dev_ms = timed_solves(hip, stream, s32, args.steps, args.warmup, n_launch)
    rec32 = s32.records()
    value = args.steps * cells / wall
    avg_kernel_us = 1e3 * float(np.mean(dev_ms)) / n_launch
    chunk_us = 1e3 * float(np.mean(dev_ms)) / n_chunks
    flop_launch = flops_per_cell_update(n_levels) * prob["nx"] * steps_per_launch
    achieved_tflops = flop_launch / (avg_kernel_us * 1e-6) / 1e12
    eff_gbs = bytes_per_cell_update(n_levels, 32) * cells / (float(np.mean(dev_ms)) * 1e-3) / 1e9
    log(f"[bench] fp32 blocked: {value:.3e} cell-updates/s, {n_launch} launch(es) of {steps_per_launch} steps "
        f"(persistent={persistent}), {avg_kernel_us:.2f} us per launch, {chunk_us:.2f} us per {depth}-step chunk")

    kname = f"k_blocked<3,float,{block},{lanes},{str(regs).lower()}" + (",strong>" if args.coupling == "strong" else ">")
    traffic = measured_traffic(kname, f"{wname}/nx{prob['nx']}", depth, steps_per_launch)
    out = {
        "metric": "cell-updates/s (FP64 plain vs FP32 batched) at stated error; p50/p99 solve latency",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wname, "field_step": args.field_step, "coupling": args.coupling,
                   "nx": prob["nx"], "n_steps": prob["n_steps"], "levels": 3,
                   "materials": len(prob["materials"]), "records": len(prob["records"]),
                   "variant": "blocked", "block": block, "depth": depth, "regs": regs, "lanes": lanes, "setup_s": t_setup,
                   "step": "one full solve of the workload"},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": PEAK["fp32_tflops"],
                     "unit": "TFLOP/s", "frac": achieved_tflops / PEAK["fp32_tflops"], "traffic": traffic,
                     # the kernels issue unpacked FP32 (packed FP32 is disabled): their own ceiling
                     "frac_of_unpacked_fp32": achieved_tflops / PEAK["fp64_tflops"],
                     "traffic_unit": "bytes per launch (HBM, counter-measured)",
                     "kernel": kname, "avg_kernel_us": avg_kernel_us, "persistent": persistent,
                     "launches_per_solve": n_launch, "steps_per_launch": steps_per_launch,
                     "chunk_us": chunk_us,
                     "flops_per_cell_update": flops_per_cell_update(n_levels),
                     "flops_per_cell_update_issued": flops_issued_per_cell_update(n_levels),
                     "cell_updates_per_launch": prob["nx"] * steps_per_launch,
                     "bytes_algorithmic_per_s": eff_gbs * 1e9},
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu

    # ---- FP64 legs ---------------------------------------------------------------------
    rec64 = None
    if not args.no_fp64:
        log("[bench] lambda3 fp64 blocked")
        s64 = mb.Solver(prob, precision=64, variant=variant, block=args.block, depth=args.depth,
                        lanes=args.lanes)
        b64, k64, r64, l64 = s64.shape()
        w64, d64 = timed_solves(hip, stream, s64, 5, 1, math.ceil(prob["n_steps"] / k64))
        rec64 = s64.records()
        s64.close()
        log("[bench] lambda3 fp64 plain (two launches per step)")
        sp = mb.Solver(prob, precision=64, variant="plain")
        t0 = time.perf_counter()
        sp.run(-1, stream)
        hip.sync()
        wp = time.perf_counter() - t0
        recp = sp.records()
        sp.close()
        same = all(np.array_equal(recp[k], rec64[k]) for k in rec64)
        ms64 = float(np.median(d64))
        out["fp64_blocked"] = {"value": cells / (ms64 * 1e-3), "unit": "cell-updates/s", "device_ms_median": ms64,
                               "block": b64, "depth": k64, "regs": r64, "lanes": l64,
                               "tflops_algorithmic": alu_tflops(n_levels, cells, ms64),
                               "alu_frac": alu_tflops(n_levels, cells, ms64) / PEAK["fp64_tflops"]}
        out["fp64_plain"] = {"value": cells / wp, "unit": "cell-updates/s", "wall_s": wp,
                             "bitwise_equal_to_fp64_blocked": bool(same)}
        out["fp32_vs_fp64_full_run_max_rel_err"] = rel_err(prob, rec32, rec64)
        out["fp32_vs_fp64_full_run_crosses_1e-4_at_step"] = crossing_step(prob, rec32, rec64, 1e-4)

    # ---- errors against the oracle: the prefix timed above, and the stored full run ----
    if cpu is not None and args.nx == 32768:
        out["error_vs_oracle_prefix"] = {"steps": n_cpu, "fp32": rel_err(prob, rec32, ref_prefix)}
        if rec64 is not None:
            out["error_vs_oracle_prefix"]["fp64"] = rel_err(prob, rec64, ref_prefix)
    full_ref = stored_lambda3_records(prob)
    if full_ref is not None:
        ref, stride = full_ref
        sub = lambda rec: {k: np.asarray(v)[stride - 1::stride] for k, v in rec.items()}  # noqa: E731
        out["error_vs_oracle_full_run"] = {"steps": prob["n_steps"], "samples_per_trace": len(next(iter(ref.values()))),
                                           "fp32": max_error(prob, sub(rec32), ref)}
        if rec64 is not None:
            out["error_vs_oracle_full_run"]["fp64"] = max_error(prob, sub(rec64), ref)
    s32.close()

    # ---- batched sweep ---------------------------------------------------------------
    if not args.no_batch:
        log("[bench] batched sweep 256 sims fp32")
        sims = W.sweep(n_sims=256, precision=32)
        bcells = sum(p["nx"] * p["n_steps"] for p in sims)
        bt = mb.Batch(sims, precision=32, variant="auto")
        bblock, bdepth, bregs, blanes = bt.shape()
        bmode = bt.run_mode()
        bt.run(stream=stream, use_graph=True)
        hip.sync()
        bt.reset(stream)
        hip.sync()
        t0 = time.perf_counter()
        bt.run(stream=stream, use_graph=True)
        hip.sync()
        tb = time.perf_counter() - t0
        beff = sum(bytes_per_cell_update(2 if k % 2 == 0 else 3, 32) * p["nx"] * p["n_steps"]
                   for k, p in enumerate(sims)) / tb / 1e9
        bflop = sum(flops_per_cell_update(2 if k % 2 == 0 else 3) * p["nx"] * p["n_steps"]
                    for k, p in enumerate(sims)) / tb / 1e12
        out["batched_sweep"] = {"tflops_algorithmic": bflop, "alu_frac": bflop / PEAK["fp32_tflops"],
                                "value": bcells / tb, "unit": "cell-updates/s", "sims": len(sims),
                                "cell_updates": bcells, "wall_s": tb, "bytes_algorithmic_per_s": beff * 1e9,
                                "block": bblock, "depth": bdepth, "regs": bregs, "lanes": blanes,
                                "launch_form": {"queue": "work-queue persistent launches of both level counts",
                                                "flags": "persistent launches with neighbour flags",
                                                "chunks": "one kernel per level count and chunk, replayed from a HIP graph"}[bmode]}
        bt.close()
        # the same sweep as one work-queue persistent launch on the tuned tile
        log("[bench] batched sweep as one work-queue launch")
        os.environ["MB_QUEUE"] = "1"
        try:
            bq = mb.Batch(sims, precision=32, variant="blocked_regs" if bregs else "blocked", block=bblock,
                          depth=bdepth, lanes=1)
        finally:
            os.environ.pop("MB_QUEUE", None)
        qmode = bq.run_mode()
        bq.run(stream=stream)
        hip.sync()
        bq.reset(stream)
        hip.sync()
        t0 = time.perf_counter()
        bq.run(stream=stream)
        hip.sync()
        tq = time.perf_counter() - t0
        bq.close()
        out["batched_sweep_one_launch"] = {"value": bcells / tq, "unit": "cell-updates/s", "wall_s": tq,
                                           "launch_form": qmode, "block": bblock, "depth": bdepth,
                                           "regs": bregs}
        if not args.no_sub32:
            out["batched_sweep_sub32"] = sweep_sub_batch(hip, stream, sims[:32], log)

    # ---- other configurations --------------------------------------------------------
    if not args.no_configs:
        out["configs"] = other_configs(hip, stream, log, sit_ref=ref_sit if cpu is not None else None)

    # ---- serving ---------------------------------------------------------------------
    if not args.no_serve:
        n_fifo = 60
        out["serving"] = run_serving(args.serve_requests, 200.0, log, first_n=n_fifo)
        out["serving_low_load"] = [run_serving(n, rate, log, first_n=n)
                                   for rate, n in ((25.0, 50), (50.0, 100), (100.0, 150))]
        full = W.serve_trace(n_requests=args.serve_requests, rate=200.0, precision=32)
        low = W.serve_trace(n_requests=50, rate=25.0, precision=32)
        out["serving_fifo_plain_fp64"] = {
            "rate_200": {**plain_fifo(full[:n_fifo], log), "trace": f"first {n_fifo} requests of the 200/s trace"},
            "rate_25": {**plain_fifo(low, log), "trace": "the 50-request 25/s trace"}}

    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
