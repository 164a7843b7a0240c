"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (relative max-norm of each recorded trace, see workloads.errors:
max |x - x_ref| / max |x_ref| per trace, the reference max-norm floored at 1e-3
for density quantities and 1 V/m for E): FP64 1e-10, FP32 1e-4.  The two-launch FP64 kernels and the
blocked FP64 kernel execute the same per-cell arithmetic, so they must agree
bit for bit whatever the tile shape.
"""
import math
import os
import sys

import numpy as np
import pytest

import paper_2005_05412_amd as mb
import workloads as W
from oracle import mb_oracle as O
from workloads.errors import trace_errors, worst

pytestmark = pytest.mark.gpu

TOL = {64: 1e-10, 32: 1e-4}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_errors(prob, got, ref):
    """name -> relative max-norm error of each recorded trace."""
    return trace_errors(prob, got, ref)


def gpu_run(prob, precision=None, variant="auto", block=0, depth=0, chunks=None, lanes=0):
    s = mb.Solver(prob, precision=precision, variant=variant, block=block, depth=depth, lanes=lanes)
    if chunks:
        for c in chunks:
            s.run(c)
    s.run()
    rec = s.records()
    s.close()
    return rec


def assert_same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k]), k


SMALL = [
    dict(seed=11, N=2, nx=37, n_steps=70, refl=(0.0, 1.0)),
    dict(seed=12, N=3, nx=150, n_steps=90, refl=(1.0, 0.0), soft=True),
    dict(seed=13, N=4, nx=61, n_steps=50, refl=(0.0, 0.0), e_noise=1e7),
    dict(seed=14, N=5, nx=45, n_steps=40, refl=(1.0, 1.0)),
    dict(seed=15, N=6, nx=33, n_steps=30, refl=(0.0, 1.0)),
    dict(seed=16, N=3, nx=1, n_steps=200, refl=(0.0, 0.0)),
    dict(seed=17, N=0, nx=80, n_steps=120, refl=(0.0, 1.0)),
    dict(seed=18, N=2, nx=3, n_steps=25, refl=(0.0, 0.0)),
    dict(seed=25, N=3, nx=120, n_steps=80, refl=(0.64, 0.3)),       # semi-transparent ends
    dict(seed=26, N=5, nx=70, n_steps=40, refl=(0.8, 0.8), e_noise=1e6),
    dict(seed=27, N=7, nx=40, n_steps=30, refl=(0.0, 1.0)),
    dict(seed=28, N=8, nx=35, n_steps=25, refl=(1.0, 0.0), e_noise=1e6),
]


def _small(case):
    kw = dict(case)
    return W.random_small(kw.pop("seed"), **kw)


@pytest.mark.parametrize("case", SMALL, ids=lambda c: f"N{c['N']}-nx{c['nx']}-s{c['seed']}")
def test_small_random_fp64_plain_and_blocked_vs_oracle(case):
    prob = _small(case)
    _say(f"case {prob['name']}")
    ref = O.run(prob)
    plain = gpu_run(prob, precision=64, variant="plain")
    errs = rel_errors(prob, plain, ref)
    assert max(errs.values()) <= TOL[64], errs
    # every tile shape, coefficient placement and split of the density update
    # over 1, 2 or 4 waves per 64 cells runs the same per-cell arithmetic
    shapes = [(64, 1, 1), (64, 7, 1), (64, 20, 1), (128, 31, 1), (192, 48, 1), (256, 32, 1), (512, 100, 1),
              (64, 7, 2), (128, 31, 2), (192, 64, 2), (256, 64, 2), (64, 20, 4), (128, 16, 4), (192, 32, 4),
              (256, 32, 4), (64, 20, 8)]
    for block, depth, lanes in shapes:
        if not mb.tile_supported(case["N"], 64, block):
            continue  # no such tile for 5 and 6 levels
        for variant in ("blocked", "blocked_regs"):
            blk = gpu_run(prob, precision=64, variant=variant, block=block, depth=depth, lanes=lanes)
            assert_same(blk, plain)


@pytest.mark.parametrize("case", SMALL[:5], ids=lambda c: f"N{c['N']}-nx{c['nx']}-s{c['seed']}")
def test_small_random_fp32_vs_oracle(case):
    prob = _small(case)
    _say(f"case {prob['name']} fp32")
    ref = O.run(prob)
    got = gpu_run(prob, precision=32, variant="blocked", block=128, depth=16)
    errs = rel_errors(prob, got, ref)
    assert max(errs.values()) <= TOL[32], errs
    # every tile shape and coefficient placement runs the same per-cell arithmetic
    for variant, block, depth, lanes in (("blocked", 64, 12, 1), ("blocked_regs", 64, 16, 1),
                                         ("blocked_regs", 256, 64, 1), ("blocked", 128, 16, 2),
                                         ("blocked_regs", 64, 16, 4), ("blocked_regs", 192, 32, 4),
                                         ("blocked", 256, 64, 4)):
        assert_same(gpu_run(prob, precision=32, variant=variant, block=block, depth=depth, lanes=lanes), got)


def test_blocked_chunking_is_invisible():
    """Splitting a run into calls of arbitrary length changes nothing (bitwise)."""
    prob = W.random_small(21, N=3, nx=300, n_steps=100, refl=(0.0, 0.0))
    _say("chunking")
    whole = gpu_run(prob, precision=64, variant="blocked", block=128, depth=12)
    split = gpu_run(prob, precision=64, variant="blocked", block=128, depth=12, chunks=[1, 7, 13, 30])
    assert_same(whole, split)


def test_read_state_matches_oracle_density():
    prob = W.random_small(22, N=3, nx=50, n_steps=40, refl=(1.0, 0.0), full_records=False)
    _say("state")
    orc = O.Oracle(prob)
    orc.run()
    s = mb.Solver(prob, precision=64)
    s.run()
    e, h, rho = s.state()
    s.close()
    assert np.max(np.abs(e - orc.e)) <= 1e-10 * np.max(np.abs(orc.e))
    assert np.max(np.abs(h[:-1] - orc.h)) <= 1e-10 * np.max(np.abs(orc.h))
    ref = orc.full_density()
    qm_cells = np.nonzero(np.abs(np.trace(ref, axis1=1, axis2=2)) > 0.5)[0]
    assert len(qm_cells) > 10
    assert np.max(np.abs(rho[qm_cells] - ref[qm_cells])) < 1e-10


def test_nonfinite_field_is_reported():
    prob = W.random_small(23, N=2, nx=40, n_steps=10, full_records=False)
    prob["records"] = [W.record("e", "e", 20, 1)]
    prob["e_init"] = np.zeros(40)
    prob["e_init"][20], prob["e_init"][21] = 1.7e308, -1.7e308   # finite, overflows in the first step
    s = mb.Solver(prob, precision=64)
    s.run()
    with pytest.raises(mb.MBError) as ex:
        s.record(0)
    assert ex.value.code == -7
    s.close()


# ---------------------------------------------------------------- benchmark configurations

def test_sit_two_level_full_fp64_and_fp32():
    """Two-level SIT, 1500 cells, 20000 steps: FP64 within 1e-10, FP32 within 1e-4."""
    prob = W.sit_2lvl()
    _say("sit oracle")
    ref = O.run(prob)
    _say("sit gpu fp64")
    got = gpu_run(prob, precision=64)
    errs = rel_errors(prob, got, ref)
    _say(f"sit fp64 errors {errs}")
    assert max(errs.values()) <= TOL[64], errs
    got32 = gpu_run(prob, precision=32)
    errs32 = rel_errors(prob, got32, ref)
    _say(f"sit fp32 errors {errs32}")
    assert max(errs32.values()) <= TOL[32], errs32


def test_lambda3_full_grid_prefix_vs_oracle():
    """Three-level Lambda medium at its full 32768-cell grid, first 600 steps."""
    prob = W.lambda3(n_steps=600, rec_interval=10)
    _say("lambda3 oracle prefix")
    ref = O.run(prob)
    got = gpu_run(prob, precision=64)
    errs = rel_errors(prob, got, ref)
    assert max(errs.values()) <= TOL[64], max(errs.values())
    got32 = gpu_run(prob, precision=32)
    errs32 = rel_errors(prob, got32, ref)
    assert max(errs32.values()) <= TOL[32], max(errs32.values())
    # the density update split over 2 or 4 waves per 64 cells gives the same bits
    base = gpu_run(prob, precision=32, variant="blocked", block=256, depth=64, lanes=1)
    for block, depth, lanes in ((256, 64, 2), (128, 32, 4), (192, 32, 4), (256, 64, 4), (512, 128, 2)):
        for variant in ("blocked", "blocked_regs"):
            _say(f"lambda3 prefix {variant} {block}/{depth} lanes {lanes}")
            assert_same(gpu_run(prob, precision=32, variant=variant, block=block, depth=depth, lanes=lanes), base)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _stored(name):
    """Oracle records written by tests/golden/make_oracle_records.py (oracle and input
    generators only)."""
    sys.path.insert(0, GOLDEN)
    from make_oracle_records import fingerprint
    d = np.load(os.path.join(GOLDEN, name))
    return d, fingerprint


def test_lambda3_full_run_vs_stored_oracle_records():
    """The Lambda workload over all 200000 steps (Alg. 1 on the full 32768-cell grid, the
    Gaussian train of Sec. 4-style drive crossing the first probes) against the oracle's
    records, every 100th step of each of the 192 traces: FP64 within 1e-10 and FP32 within
    1e-4 per trace.
    The records see the drive: an undriven run differs from them by far more than 1e-4 on
    at least 20 probes."""
    d, fingerprint = _stored("oracle_lambda3.npz")
    prob = W.lambda3()
    assert str(d["lambda3/fingerprint"]) == fingerprint(prob), "generators changed since the records were written"
    stride = int(d["lambda3/stride"])
    ref = {r["name"]: d["lambda3/" + r["name"]] for r in prob["records"]}
    sub = lambda rec: {k: np.asarray(v)[stride - 1::stride] for k, v in rec.items()}  # noqa: E731
    _say("lambda3 full fp64 vs stored oracle")
    got = sub(gpu_run(prob, precision=64))
    errs = rel_errors(prob, got, ref)
    _say(f"lambda3 full fp64 worst {worst(errs)}")
    assert max(errs.values()) <= TOL[64], worst(errs)
    got32 = sub(gpu_run(prob, precision=32))
    errs32 = rel_errors(prob, got32, ref)
    _say(f"lambda3 full fp32 worst {worst(errs32)}")
    assert max(errs32.values()) <= TOL[32], worst(errs32)
    quiet = dict(prob)
    quiet["sources"] = [dict(src, amp=0.0) for src in prob["sources"]]
    undriven = rel_errors(prob, sub(gpu_run(quiet, precision=64)), ref)
    driven_probes = {name.split("@")[-1] for name, e in undriven.items() if e > 1e-4}
    assert len(driven_probes) >= 20, sorted(driven_probes)


def _uneven_sweep(n_sims, n_steps0, step, nx_range, precision=32):
    """Sweep members (even index two levels, odd three) of uneven lengths."""
    sims = W.sweep(n_sims=n_sims, n_steps=n_steps0 + step * n_sims, precision=precision, nx_range=nx_range)
    for k, p in enumerate(sims):
        p["n_steps"] = n_steps0 + step * k
    return sims


def _batch_records(sims, precision, queue, **shape):
    if queue:
        os.environ["MB_QUEUE"] = "1"
    try:
        b = mb.Batch([dict(p, precision=precision) for p in sims], precision=precision, **shape)
        mode = b.run_mode()
        b.run(use_graph=False)
        recs = [b.records(k) for k in range(len(sims))]
        b.close()
    finally:
        os.environ.pop("MB_QUEUE", None)
    return mode, recs


@pytest.mark.parametrize("precision", [32, 64])
def test_mixed_level_uneven_batch_in_one_work_queue_launch(precision):
    """Many uneven-length simulations of two and three levels in one persistent launch:
    the batch's full chunks run as one work-queue launch (each workgroup takes (chunk,
    tile) items of either level count until none is left), with results bit for bit
    those of one launch per chunk and level count; two members (one of each level count)
    against the oracle: FP64 within 1e-10, FP32 within 1e-4 per trace."""
    sims = _uneven_sweep(24, 1000, 90, (300, 4000))
    _say(f"work-queue batch fp{precision}")
    shape = dict(block=256, depth=32, lanes=1)
    mode_q, rec_q = _batch_records(sims, precision, True, **shape)
    mode_c, rec_c = _batch_records(sims, precision, False, **shape)
    assert (mode_q, mode_c) == ("queue", "chunks")
    for a, b in zip(rec_q, rec_c):
        assert_same(a, b)
    small = sorted(range(len(sims)), key=lambda k: sims[k]["nx"] * sims[k]["n_steps"])
    for k in (next(k for k in small if k % 2 == 0), next(k for k in small if k % 2 == 1)):
        ref = O.run(dict(sims[k], precision=64))
        errs = trace_errors(sims[k], rec_q[k], ref)
        _say(f"work-queue member {k} nx={sims[k]['nx']} steps={sims[k]['n_steps']} {worst(errs)}")
        assert max(errs.values()) <= TOL[precision], (k, worst(errs))


def test_single_grid_beyond_residency_takes_the_work_queue():
    """A three-level grid of 3e6 cells has more 256-cell tiles than the device holds at
    once: the neighbour-flag persistent form does not apply, the work-queue form does,
    and gives the bits of one launch per chunk."""
    prob = W.lambda3(nx=3_000_000, n_steps=256, precision=32)
    prob["records"] = prob["records"][:12]
    _say("work-queue single grid")
    out = {}
    for queue in (True, False):
        if queue:
            os.environ["MB_QUEUE"] = "1"
        try:
            s = mb.Solver(prob, precision=32, variant="blocked", block=256, depth=32, lanes=1)
            mode = s.persistent()
            s.run()
            out[queue] = (mode, s.records())
            s.close()
        finally:
            os.environ.pop("MB_QUEUE", None)
    assert out[True][0] and not out[False][0]
    assert_same(out[True][1], out[False][1])


@pytest.mark.parametrize("precision", [64, 32])
def test_sweep_members_full_length_vs_stored_oracle_records(precision):
    """The 256-member sweep as one batch; its 8 seeded spot-check members over their full
    50000 steps against the oracle's records (E and populations at both probes every 50
    steps): FP64 within 1e-10 and FP32 within 1e-4 per trace; both probes of every member
    see the drive (an undriven oracle-free check: the records' E traces are far from zero)."""
    d, fingerprint = _stored("oracle_sweep_picks.npz")
    sims = W.sweep(n_sims=256, precision=32)
    picks = np.random.default_rng(W.SEED_BASE + 3).choice(256, 8, replace=False)
    b = mb.Batch([dict(p, precision=precision) for p in sims], precision=precision)
    _say(f"sweep batch fp{precision} vs stored oracle")
    b.run(use_graph=True)
    for k in picks:
        k = int(k)
        p = sims[k]
        assert str(d[f"sweep{k}/fingerprint"]) == fingerprint(p), k
        ref = {r["name"]: d[f"sweep{k}/" + r["name"]] for r in p["records"]}
        errs = trace_errors(p, b.records(k), ref)
        _say(f"sweep member {k} nx={p['nx']} fp{precision} worst {worst(errs)}")
        assert max(errs.values()) <= TOL[precision], (k, worst(errs))
        for r in p["records"]:
            if r["quantity"] == "e":
                assert np.max(np.abs(ref[r["name"]])) > 1e3, (k, r["name"])   # the pulse reached the probe
    b.close()


def test_lambda3_full_length_blocked_equals_plain_and_invariants():
    """Full 200000 steps: blocked FP64 == two-launch FP64 bit for bit; populations valid."""
    prob = W.lambda3()
    _say("lambda3 full plain")
    plain = gpu_run(prob, precision=64, variant="plain")
    _say("lambda3 full blocked")
    blk = gpu_run(prob, precision=64, variant="blocked")
    assert_same(blk, plain)
    for k in range(64):
        names = [r["name"] for r in prob["records"][3 * k: 3 * k + 3]]
        pops = np.array([blk[n] for n in names])
        assert np.max(np.abs(pops.sum(axis=0) - 1.0)) < 1e-12
        assert pops.min() > -1e-10 and pops.max() < 1 + 1e-10


# ---------------------------------------------------------------- batching and serving

def _mixed_batch(n=6, n_steps=1600, precision=32):
    rng = np.random.default_rng(5)
    probs = []
    for k in range(n):
        nx = int(rng.integers(50, 500))
        probs.append(W.sweep_sim(k, rng, nx=nx, n_steps=n_steps + 37 * k, precision=precision,
                                 rec_interval=5))
    return probs


@pytest.mark.parametrize("precision", [64, 32])
def test_batch_equals_individual_runs(precision):
    probs = _mixed_batch(precision=precision)
    _say(f"batch {precision}")
    b = mb.Batch(probs, precision=precision, block=128, depth=16, lanes=2)
    b.run(use_graph=True)
    for k, p in enumerate(probs):
        alone = gpu_run(p, precision=precision, variant="blocked", block=256, depth=32)
        assert_same(b.records(k), alone)
    b.close()
    if precision == 64:
        for k in (0, 1):
            ref = O.run(probs[k])
            b2 = mb.Batch(probs, precision=64, block=128, depth=16)
            b2.run(use_graph=False)
            errs = rel_errors(probs[k], b2.records(k), ref)
            b2.close()
            assert max(errs.values()) <= TOL[64], errs


class _persist:
    """Engines created inside the block run every chunk as its own launch (MB_PERSIST=0) or not."""

    def __init__(self, on):
        self.on = on

    def __enter__(self):
        import os
        self.old = os.environ.get("MB_PERSIST")
        os.environ["MB_PERSIST"] = "1" if self.on else "0"

    def __exit__(self, *exc):
        import os
        if self.old is None:
            os.environ.pop("MB_PERSIST", None)
        else:
            os.environ["MB_PERSIST"] = self.old


def test_persistent_launch_equals_relaunches():
    """Chunks chained in one launch by neighbour flags give the bits of one launch per chunk."""
    prob = _small(SMALL[1])                      # 3 levels, 150 cells, soft source
    prob["n_steps"] = 400
    for precision, variant, block, depth, lanes in ((64, "blocked", 64, 16, 1), (64, "blocked_regs", 128, 16, 2),
                                                    (32, "blocked_regs", 192, 32, 4), (32, "blocked", 64, 8, 4),
                                                    (64, "blocked", 256, 64, 2)):
        _say(f"persistent {precision} {variant} {block}/{depth}/{lanes}")
        with _persist(False):
            ref = gpu_run(prob, precision=precision, variant=variant, block=block, depth=depth, lanes=lanes)
        with _persist(True):
            got = gpu_run(prob, precision=precision, variant=variant, block=block, depth=depth, lanes=lanes,
                          chunks=[5, 100])
        assert_same(got, ref)
    # one level count, uneven lengths and step counts: simulations finish in different chunks
    rng = np.random.default_rng(9)
    probs = [W.sweep_sim(k, rng, nx=int(rng.integers(100, 900)), n_steps=700 + 61 * k, precision=32,
                         rec_interval=5) for k in range(0, 12, 2)]    # even members: two levels
    _say(f"persistent batch of {len(probs)}")
    with _persist(True):
        b = mb.Batch(probs, precision=32, block=128, depth=32, lanes=2)
        b.run(use_graph=False)
        got = [b.records(k) for k in range(len(probs))]
        b.close()
    with _persist(False):
        for k, p in enumerate(probs):
            assert_same(got[k], gpu_run(p, precision=32, variant="blocked", block=128, depth=32, lanes=2))


def test_server_results_equal_alone():
    """Requests admitted while others run give the same records as solo runs (two of them
    with the Cayley field step, which run as a kernel group of their own, and a six-level
    one with a drive), and three of them, the six-level one included, match the oracle."""
    probs = _mixed_batch(n=8, n_steps=300, precision=32)
    for k in (2, 5):
        probs[k]["field_step"] = "cayley"
    six = W.qcl6(nx=240, n_steps=300, precision=32, rec_interval=5)
    six["refl"] = (0.0, 0.0)
    six["sources"] = [W.source("gauss", 0.0, 1e6, 3e12, 5.0, 1.0 / 500e-15)]
    probs.insert(4, six)
    _say("server")
    srv = mb.Server(hbm_budget=256 << 20, max_slots=3, precision=32, chunk_steps=16)
    tickets = [srv.submit(p, arrival_s=0.002 * k) for k, p in enumerate(probs)]
    srv.start()
    srv.drain(timeout_s=120)
    for t, p in zip(tickets, probs):
        st = srv.status(t)
        assert st[0] == 2, st
        alone = gpu_run(p, precision=32, variant="blocked", block=256, depth=32)
        for k, r in enumerate(p["records"]):
            assert np.array_equal(srv.record(t, k), alone[r["name"]]), r["name"]
    for i in (0, 3, 4):                      # two-level, three-level (Cayley-free), six-level
        p, t = probs[i], tickets[i]
        got = {r["name"]: srv.record(t, k) for k, r in enumerate(p["records"])}
        errs = rel_errors(p, got, O.run(p))
        _say(f"server vs oracle {p['name']} {max(errs.values()):.2e}")
        assert max(errs.values()) <= TOL[32], (p["name"], errs)
    cu, busy, chunks = srv.stats()
    assert cu == sum(p["nx"] * p["n_steps"] for p in probs)
    polled = srv.poll(capacity=5) + srv.poll()
    assert sorted(polled) == sorted(tickets) and srv.poll() == []
    srv.close()


def test_server_budget_and_cancel():
    p = _mixed_batch(n=1, n_steps=100, precision=32)[0]
    srv = mb.Server(hbm_budget=1 << 12, max_slots=2, precision=32, chunk_steps=16)
    with pytest.raises(mb.MBError) as ex:
        srv.submit(p)
    assert ex.value.code == -5
    srv.close()
    srv = mb.Server(hbm_budget=64 << 20, max_slots=1, precision=32, chunk_steps=16)
    t1 = srv.submit(p, 0.0)
    big = dict(p)
    big["n_steps"] = 200000
    t2 = srv.submit(big, 0.0)
    srv.cancel(t2)
    srv.start()
    srv.drain(timeout_s=60)
    assert srv.status(t1)[0] == 2
    assert srv.status(t2)[0] == 3
    assert sorted(srv.poll()) == sorted([t1, t2])      # done and cancelled both reported once
    assert srv.poll() == []
    srv.close()


@pytest.mark.parametrize("n,seed", [(2, 71), (3, 72), (5, 73)])
def test_explicit_lindblad_ops_vs_oracle(n, seed):
    """Materials described by explicit Lindblad operators (eq:lindbladdiss) instead of rates:
    FP64 within 1e-10 and FP32 within 1e-4 of the oracle; blocked == two-launch bitwise."""
    prob = W.random_small(seed, N=n, nx=70, n_steps=60, refl=(0.0, 1.0))
    rng = np.random.default_rng(seed)
    for m in prob["materials"]:
        if m["qm"] is not None:
            m["qm"] = dict(m["qm"], lindblad_ops=[(rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))
                                                  * np.sqrt(1e12 / n) for _ in range(3)])
    _say(f"lindblad ops {prob['name']}")
    ref = O.run(prob)
    plain = gpu_run(prob, precision=64, variant="plain")
    errs = rel_errors(prob, plain, ref)
    assert max(errs.values()) <= TOL[64], errs
    assert_same(gpu_run(prob, precision=64, variant="blocked", block=128, depth=16), plain)
    errs32 = rel_errors(prob, gpu_run(prob, precision=32, variant="blocked", block=64, depth=16), ref)
    assert max(errs32.values()) <= TOL[32], errs32


def test_table_sources_vs_oracle():
    """Sampled-waveform sources (a hard one shorter than the run and a soft one) drive a
    random three-level device: FP64 within 1e-10 and FP32 within 1e-4 of the oracle."""
    prob = W.random_small(81, N=3, nx=90, n_steps=120, refl=(0.0, 1.0))
    rng = np.random.default_rng(81)
    amp = max(abs(s["amp"]) for s in prob["sources"]) if prob["sources"] else 1e9
    # the soft source sits half way between nodes 44 and 45: both sides take the even node
    prob["sources"] = [W.table_source(0.0, amp * np.sin(0.3 * np.arange(80)) * np.exp(-np.arange(80) / 40.0)),
                       W.table_source(W.node_x(prob["length"], 90, 44.5), 0.1 * amp * rng.normal(size=121),
                                      hard=False)]
    _say("table sources")
    ref = O.run(prob)
    plain = gpu_run(prob, precision=64, variant="plain")
    errs = rel_errors(prob, plain, ref)
    assert max(errs.values()) <= TOL[64], errs
    assert_same(gpu_run(prob, precision=64, variant="blocked", block=128, depth=16), plain)
    errs32 = rel_errors(prob, gpu_run(prob, precision=32, variant="blocked", block=128, depth=16), ref)
    assert max(errs32.values()) <= TOL[32], errs32


@pytest.mark.parametrize("noise,precision", [(5e11, 64), (3e10, 32)])
def test_large_field_phases_vs_oracle(noise, precision):
    """Field phases far beyond the series range (up to ~12 rad per step in FP64, ~0.7 in
    FP32, past both precisions' series limits) take the range-reduced path: FP64 within
    1e-10, FP32 within 1e-4 of the oracle; FP64 blocked == two-launch bitwise."""
    prob = W.random_small(91, N=3, nx=50, n_steps=40, e_noise=noise, refl=(1.0, 1.0))
    kap = max(np.abs(mb.plan_material(prob, k)["kappa"]).max() for k in (1, 2))
    angle = kap * np.abs(prob["e_init"]).max()
    assert angle > (3.0 if precision == 64 else 0.5), angle
    _say(f"large phases {precision}: {angle:.2f} rad")
    ref = O.run(prob)
    if precision == 64:
        got = gpu_run(prob, precision=64, variant="plain")
        assert_same(gpu_run(prob, precision=64, variant="blocked", block=64, depth=8), got)
    else:
        got = gpu_run(prob, precision=32, variant="blocked", block=64, depth=8)
    errs = rel_errors(prob, got, ref)
    assert max(errs.values()) <= TOL[precision], errs


def test_library_drawn_initial_field():
    """Without an e_init array the library draws E_m = c + A (2 u_m - 1) from SplitMix64
    itself: the same initial field and the same run, bit for bit, as the array drawn by the
    input generator (an independent SplitMix64)."""
    base = W.random_small(95, N=3, nx=80, n_steps=50, refl=(0.0, 1.0))
    spec = {"const": 2e6, "noise": 3e8, "seed": 12345}
    lib = dict(base, e_init=None, e_field=spec)
    arr = dict(base, e_init=spec["const"] + spec["noise"] * (2.0 * W.splitmix64_uniform(spec["seed"], 80) - 1.0))
    _say("library-drawn initial field")
    for precision, variant in ((64, "plain"), (32, "blocked")):
        shape = dict(block=64, depth=16) if variant == "blocked" else {}
        a = mb.Solver(lib, precision=precision, variant=variant, **shape)
        b = mb.Solver(arr, precision=precision, variant=variant, **shape)
        assert np.array_equal(a.state(3)[0], b.state(3)[0])
        a.run()
        b.run()
        assert_same(a.records(), b.records())
        a.close()
        b.close()


def test_degenerate_runs():
    """No steps, a record period longer than the run, run(0), and such members in a batch:
    empty records like the oracle's, and the other members unchanged."""
    p0 = W.random_small(31, N=3, nx=40, n_steps=0)
    p1 = W.random_small(32, N=2, nx=40, n_steps=5, rec_interval=10)
    p2 = W.random_small(33, N=3, nx=90, n_steps=40)
    _say("degenerate")
    for p in (p0, p1):
        ref = O.run(p)
        for precision, variant in ((64, "plain"), (64, "blocked"), (32, "blocked")):
            got = gpu_run(p, precision=precision, variant=variant)
            for k in ref:
                assert got[k].size == 0 and np.asarray(ref[k]).size == 0, k
    s = mb.Solver(p2, precision=64, variant="blocked", block=128, depth=16)
    s.run(0)
    s.run(0)
    assert s.steps_done == 0
    s.run()
    assert_same(s.records(), gpu_run(p2, precision=64, variant="blocked", block=128, depth=16))
    s.close()
    b = mb.Batch([p0, p2, p1], precision=32, block=128, depth=16)
    b.run(use_graph=True)
    assert_same(b.records(1), gpu_run(p2, precision=32, variant="blocked", block=128, depth=16))
    for k in (0, 2):
        assert all(v.size == 0 for v in b.records(k).values())
    b.close()


def test_caller_workspace():
    """mb_setup into caller-owned device memory (hipMalloc'ed here, filled with 0xFF) gives
    the same records as library-allocated memory; a workspace that is too small or
    misaligned is refused before any device work."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    prob = W.random_small(12, N=3, nx=150, n_steps=90, refl=(1.0, 0.0), soft=True)
    _say("workspace")
    for precision, variant in ((64, "plain"), (32, "blocked")):
        need = mb.workspace_bytes(prob, precision=precision, variant=variant)
        shape = dict(block=128, depth=16) if variant == "blocked" else {}
        ref = gpu_run(prob, precision=precision, variant=variant, **shape)
        ptr = ctypes.c_void_p()
        assert hip.hipMalloc(ctypes.byref(ptr), ctypes.c_size_t(need + 512)) == 0
        try:
            assert ptr.value % 256 == 0
            assert hip.hipMemset(ptr, 0xFF, ctypes.c_size_t(need + 512)) == 0
            assert hip.hipDeviceSynchronize() == 0
            s = mb.Solver(prob, precision=precision, variant=variant, workspace=(ptr.value, need), **shape)
            s.run()
            assert_same(s.records(), ref)
            s.close()
            for bad in ((ptr.value, need - 256), (ptr.value + 64, need + 256)):
                with pytest.raises(mb.MBError) as ex:
                    mb.Solver(prob, precision=precision, variant=variant, workspace=bad, **shape)
                assert ex.value.code == -1
        finally:
            assert hip.hipDeviceSynchronize() == 0
            hip.hipFree(ptr)


def test_reset_and_graph_replay_reproduce_the_run():
    """mb_reset restores the initial state; the replayed graph gives identical records."""
    prob = W.random_small(24, N=2, nx=400, n_steps=300, refl=(0.0, 0.0), full_records=False)
    prob["records"] = [W.record("e", "e", 200, 3), W.record("inv", "inv", 150, 3, 0, 1)]
    s = mb.Solver(prob, precision=32, variant="blocked", block=128, depth=16)
    s.run()
    first = s.records()
    for _ in range(2):
        s.reset()
        s.run()
        again = s.records()
        assert_same(first, again)
    s.close()


def test_qcl6_full_grid_prefix_vs_oracle():
    """Six-level QCL-like cavity (8192 cells, PEC ends, noise start): first 600 steps.

    FP64 within 1e-10 and FP32 within 1e-4 per trace."""
    prob = W.qcl6(n_steps=600)
    _say("qcl6 oracle prefix")
    ref = O.run(prob)
    got = gpu_run(prob, precision=64)
    errs = rel_errors(prob, got, ref)
    _say(f"qcl6 fp64 {errs}")
    assert max(errs.values()) <= TOL[64], errs
    got32 = gpu_run(prob, precision=32)
    errs32 = rel_errors(prob, got32, ref)
    _say(f"qcl6 fp32 {errs32}")
    assert max(errs32.values()) <= TOL[32], errs32
    base = gpu_run(prob, precision=32, variant="blocked", block=256, depth=64, lanes=1)
    for block, depth, lanes in ((128, 32, 2), (64, 16, 4), (64, 16, 8)):
        _say(f"qcl6 prefix {block}/{depth} lanes {lanes}")
        assert_same(gpu_run(prob, precision=32, variant="blocked", block=block, depth=depth, lanes=lanes), base)


def test_qcl5_comb_prefix_vs_oracle():
    """The paper's five-level QCL comb example (8192 cells, R = 0.8 mirrors, noise start):
    first 600 steps against the oracle, FP64 within 1e-10 and FP32 within 1e-4 per trace;
    the density update split over 4 and 8 waves gives the same bits."""
    prob = W.qcl5_comb(n_steps=600)
    _say("qcl5 oracle prefix")
    ref = O.run(prob)
    got = gpu_run(prob, precision=64)
    errs = rel_errors(prob, got, ref)
    _say(f"qcl5 fp64 {errs}")
    assert max(errs.values()) <= TOL[64], errs
    got32 = gpu_run(prob, precision=32)
    errs32 = rel_errors(prob, got32, ref)
    _say(f"qcl5 fp32 {errs32}")
    assert max(errs32.values()) <= TOL[32], errs32
    base = gpu_run(prob, precision=32, variant="blocked", block=256, depth=64, lanes=1)
    for block, depth, lanes in ((128, 32, 2), (64, 16, 4)):
        assert_same(gpu_run(prob, precision=32, variant="blocked", block=block, depth=depth, lanes=lanes), base)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_anharmonic_ladder_vs_oracle(n):
    """The level-count benchmark system of Sec. 4.3 (anharmonic ladder), 300 cells x 400
    steps: FP64 within 1e-10, FP32 within 1e-4, every split of the density update the same."""
    prob = W.ladder(n, nx=300, n_steps=400, rec_interval=4)
    _say(f"ladder {n}")
    ref = O.run(prob)
    got = gpu_run(prob, precision=64)
    assert max(rel_errors(prob, got, ref).values()) <= TOL[64]
    got32 = gpu_run(prob, precision=32, variant="blocked", block=128, depth=16, lanes=1)
    errs32 = rel_errors(prob, got32, ref)
    assert max(errs32.values()) <= TOL[32], errs32
    for block, depth, lanes in ((128, 16, 2), (64, 8, 4), (64, 8, 8)):
        assert_same(gpu_run(prob, precision=32, variant="blocked", block=block, depth=depth, lanes=lanes), got32)


@pytest.mark.parametrize("n", [7, 8])
def test_ladder_seven_and_eight_levels_vs_oracle(n):
    """The level-count benchmark of Sec. 4.3 (any N >= 2) beyond six levels: the anharmonic
    ladder at 7 and 8 levels, 300 cells x 400 steps, in the block form (the ladder's) and
    forced into the general form: FP64 within 1e-10 and FP32 within 1e-4 per trace; both
    built tiles (128 and 256 cells, one wave per 64 cells) bit for bit the same, a request
    for two waves per 64 cells runs the one built, and the two-launch FP64 kernel matches
    the blocked one bit for bit."""
    prob = W.ladder(n, nx=300, n_steps=400, rec_interval=4)
    _say(f"ladder {n}")
    assert mb.tile_supported(n, 32, 128) and mb.tile_supported(n, 64, 256)
    assert not mb.tile_supported(n, 32, 64) and not mb.tile_supported(n, 32, 128, lanes=2)
    ref = O.run(prob)
    for form in ("block", "general"):
        if form == "general":
            os.environ["MB_BLOCK_FORM"] = "0"
        try:
            assert mb.plan_material(prob, 1)["block"] == (form == "block")
            for precision in (64, 32):
                base = gpu_run(prob, precision=precision, variant="blocked", block=128, depth=16, lanes=1)
                errs = rel_errors(prob, base, ref)
                _say(f"ladder {n} {form} fp{precision} {worst(errs)}")
                assert max(errs.values()) <= TOL[precision], (form, precision, worst(errs))
                assert_same(gpu_run(prob, precision=precision, variant="blocked", block=256, depth=32, lanes=1), base)
                assert_same(gpu_run(prob, precision=precision, variant="blocked", block=128, depth=16, lanes=2), base)
                if precision == 64:
                    assert_same(gpu_run(prob, precision=64, variant="plain"), base)
        finally:
            os.environ.pop("MB_BLOCK_FORM", None)


@pytest.mark.parametrize("n", [2, 3, 6])
def test_field_free_medium_stays_field_free(n):
    """A medium left in its stationary ground state with no source produces no polarization
    (the field factor is the identity at E = 0): E, recorded over the whole grid, stays
    exactly zero in FP64 and FP32, as in the oracle, and the populations stay put."""
    prob = W.ladder(n, nx=300, n_steps=200, rec_interval=10)
    prob["sources"] = []
    prob["records"] = [W.record("e_all", "e", -1, 10), W.record("pop0", "pop", 150, 10, i=0, j=0)]
    for precision in (64, 32):
        got = gpu_run(prob, precision=precision)
        assert not np.any(got["e_all"]), precision
        assert np.max(np.abs(got["pop0"] - 1.0)) <= (1e-15 if precision == 64 else 1e-7)


@pytest.mark.parametrize("n", [3, 6])
def test_block_and_general_forms_vs_oracle(n):
    """The ladder's tables are block structured (real dipoles, diagonal H0, rate-form
    relaxation), so its kernels take the block form; forced into the general form
    (MB_BLOCK_FORM=0) the same solve also matches the oracle: FP64 within 1e-10 and FP32
    within 1e-4 per trace in both forms, each form bit for bit the same on every tile
    shape.  The QCL-like material (tunnelling couplings in H0) takes the general form."""
    prob = W.ladder(n, nx=300, n_steps=400, rec_interval=4)
    assert mb.plan_material(prob, 1)["block"]
    assert not mb.plan_material(W.qcl6(nx=64, n_steps=10), 0)["block"]
    ref = O.run(prob)
    for form in ("block", "general"):
        if form == "general":
            os.environ["MB_BLOCK_FORM"] = "0"
        try:
            assert mb.plan_material(prob, 1)["block"] == (form == "block")
            for precision in (64, 32):
                base = gpu_run(prob, precision=precision, variant="blocked", block=128, depth=16, lanes=1)
                errs = rel_errors(prob, base, ref)
                _say(f"ladder {n} {form} fp{precision} {worst(errs)}")
                assert max(errs.values()) <= TOL[precision], (form, precision, worst(errs))
                for block, depth, lanes in ((64, 8, 2), (64, 8, 4), (192, 32, 1)):
                    assert_same(gpu_run(prob, precision=precision, variant="blocked", block=block, depth=depth,
                                        lanes=lanes), base)
        finally:
            os.environ.pop("MB_BLOCK_FORM", None)


STRONG = [
    dict(seed=41, N=2, nx=60, n_steps=80, refl=(0.0, 1.0)),
    dict(seed=42, N=3, nx=150, n_steps=90, refl=(0.64, 0.0), soft=True),
    dict(seed=43, N=5, nx=45, n_steps=40, refl=(1.0, 1.0), e_noise=1e7),
    dict(seed=44, N=3, nx=1, n_steps=200, refl=(0.0, 0.0)),
]


@pytest.mark.parametrize("case", STRONG, ids=lambda c: f"N{c['N']}-nx{c['nx']}-s{c['seed']}")
def test_strong_coupling_vs_oracle(case):
    """Strong coupling (rho at the times of E, Sec. 2.2): FP64 within 1e-10 and FP32 within
    1e-4 of the oracle, whose field iteration runs to convergence; every tile shape the same."""
    kw = dict(case)
    prob = W.random_small(kw.pop("seed"), **kw)
    prob["coupling"] = "strong"
    _say(f"strong {prob['name']}")
    ref = O.run(prob)
    got = gpu_run(prob, precision=64, variant="blocked", block=128, depth=16)
    errs = rel_errors(prob, got, ref)
    assert max(errs.values()) <= TOL[64], errs
    for block, depth in ((64, 7), (256, 32), (512, 100)):
        if mb.tile_supported(case["N"], 64, block):
            assert_same(gpu_run(prob, precision=64, variant="blocked", block=block, depth=depth), got)
    got32 = gpu_run(prob, precision=32, variant="blocked", block=128, depth=16)
    errs32 = rel_errors(prob, got32, ref)
    assert max(errs32.values()) <= TOL[32], errs32
    # three-level FP32 256-cell tiles also run with register coefficients: same bits
    assert_same(gpu_run(prob, precision=32, variant="blocked_regs", block=256, depth=32), got32)


def test_strong_coupling_dense_medium():
    """Strong coupling in a medium 4000 times denser than the random cases: there the field
    update depends on the polarization enough (the oracle's fixed-point iteration contracts
    by about 1e-3 per pass) that the FP64 bound of 1e-10 needs the Newton steps' derivative.
    An FP64 emulation on the host of the same warm start (previous polarization current)
    differs from the converged oracle by 1.3e-4 / 1.2e-7 / 1.2e-10 (worst trace) after one /
    two / three fixed-point passes, and by 1.7e-6 / 2e-15 after one / two Newton steps (the
    FP32 and FP64 kernels' counts)."""
    prob = W.random_small(42, N=3, nx=150, n_steps=90, refl=(0.64, 0.0), soft=True)
    prob["coupling"] = "strong"
    for m in prob["materials"]:
        if m.get("qm"):
            m["qm"]["n3d"] *= 4000.0
    _say("strong dense")
    ref = O.run(prob)
    for block, depth in ((128, 16), (256, 32)):
        errs = rel_errors(prob, gpu_run(prob, precision=64, variant="blocked", block=block, depth=depth), ref)
        assert max(errs.values()) <= TOL[64], worst(errs)
    errs32 = rel_errors(prob, gpu_run(prob, precision=32, variant="blocked_regs", block=256, depth=32), ref)
    assert max(errs32.values()) <= TOL[32], worst(errs32)


def test_strong_coupling_sit_prefix_and_mixed_batch():
    """Two-level SIT with strong coupling, first 4000 steps against the oracle; a batch that
    mixes weakly and strongly coupled simulations gives each one's solo records."""
    prob = W.sit_2lvl(n_steps=4000)
    prob["coupling"] = "strong"
    _say("strong sit")
    ref = O.run(prob)
    errs = rel_errors(prob, gpu_run(prob, precision=64), ref)
    assert max(errs.values()) <= TOL[64], errs
    errs32 = rel_errors(prob, gpu_run(prob, precision=32), ref)
    assert max(errs32.values()) <= TOL[32], errs32
    probs = _mixed_batch(n=4, n_steps=500, precision=64)
    for k in (1, 2):
        probs[k]["coupling"] = "strong"
    b = mb.Batch(probs, precision=64, block=128, depth=16)
    b.run(use_graph=True)
    for k, p in enumerate(probs):
        assert_same(b.records(k), gpu_run(p, precision=64, variant="blocked", block=256, depth=32))
    b.close()


CAYLEY = [
    dict(seed=11, N=2, nx=37, n_steps=70, refl=(0.0, 1.0)),
    dict(seed=12, N=3, nx=150, n_steps=90, refl=(1.0, 0.0), soft=True),
    dict(seed=14, N=5, nx=45, n_steps=40, refl=(1.0, 1.0)),
    dict(seed=15, N=6, nx=33, n_steps=30, refl=(0.0, 1.0)),
    dict(seed=16, N=3, nx=1, n_steps=200, refl=(0.0, 0.0)),
]


@pytest.mark.parametrize("case", CAYLEY, ids=lambda c: f"N{c['N']}-nx{c['nx']}-s{c['seed']}")
def test_cayley_field_step_vs_oracle(case):
    """Field part by the Cayley approximant: FP64 within 1e-10 and FP32 within 1e-4 of the
    oracle's Cayley run (which differs from the exact field step by 1e-7 and more on these
    cases, so the tolerance tells the two apart); every tile shape, coefficient placement and
    launch form the same bits; with strong coupling too."""
    prob = _small(case)
    prob["field_step"] = "cayley"
    _say(f"cayley {prob['name']}")
    ref = O.run(prob)
    plain = gpu_run(prob, precision=64, variant="plain")
    errs = rel_errors(prob, plain, ref)
    assert max(errs.values()) <= TOL[64], errs
    for block, depth, lanes in ((64, 7, 1), (128, 31, 1), (192, 48, 2), (256, 32, 4), (64, 20, 8)):
        assert_same(gpu_run(prob, precision=64, variant="blocked", block=block, depth=depth, lanes=lanes), plain)
    got32 = gpu_run(prob, precision=32, variant="blocked", block=128, depth=16)
    errs32 = rel_errors(prob, got32, ref)
    assert max(errs32.values()) <= TOL[32], errs32
    assert_same(gpu_run(prob, precision=32, variant="blocked", block=64, depth=16, lanes=4), got32)
    assert_same(gpu_run(prob, precision=32, variant="blocked_regs", block=128, depth=16), got32)
    # register coefficients and persistent launches (one wave per 64 cells): the same bits
    for variant in ("blocked", "blocked_regs"):
        with _persist(False):
            ref64 = gpu_run(prob, precision=64, variant=variant, block=64, depth=16)
        assert_same(ref64, plain)
        with _persist(True):
            s = mb.Solver(prob, precision=64, variant=variant, block=64, depth=16, lanes=1)
            assert s.persistent() == (prob["n_steps"] // 16 >= 2)
            s.run()
            assert_same(s.records(), plain)
            s.close()
    prob["coupling"] = "strong"
    ref = O.run(prob)
    errs = rel_errors(prob, gpu_run(prob, precision=64, variant="blocked", block=128, depth=16), ref)
    assert max(errs.values()) <= TOL[64], errs


def test_cayley_sit_prefix_tuned_and_batched():
    """Two-level SIT, first 4000 steps, with the Cayley field step through the tuned (auto)
    shape in FP64 and FP32, and a batch that mixes exact and Cayley members."""
    prob = W.sit_2lvl(n_steps=4000)
    prob["field_step"] = "cayley"
    _say("cayley sit")
    ref = O.run(prob)
    got = gpu_run(prob, precision=64)
    errs = rel_errors(prob, got, ref)
    assert max(errs.values()) <= TOL[64], errs
    errs32 = rel_errors(prob, gpu_run(prob, precision=32), ref)
    assert max(errs32.values()) <= TOL[32], errs32
    probs = _mixed_batch(n=4, n_steps=500, precision=32)
    for k in (0, 3):
        probs[k]["field_step"] = "cayley"
    b = mb.Batch(probs, precision=32)
    b.run(use_graph=True)
    for k, p in enumerate(probs):
        assert_same(b.records(k), gpu_run(p, precision=32, variant="blocked", block=256, depth=32))
    b.close()

