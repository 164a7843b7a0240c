"""Python binding of libmbhip.so, the MI355X Maxwell-Bloch library.

Argument marshalling only: every step of the solve runs in the HIP kernels
behind the C ABI declared in ``include/mb.h``.  The binding converts the
problem descriptions of the ``workloads`` package (plain dicts of numbers and
numpy arrays) into the ABI's structs and returns records as numpy arrays.
It raises ``MBError`` when the library reports an error and
``LibraryMissing`` when the shared library has not been built; there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmbhip.so")

MB_OK = 0
MB_WARN_NOT_CP = 1
ERRORS = {-1: "MB_ERR_ARG", -2: "MB_ERR_CFL", -3: "MB_ERR_UNSUPPORTED", -4: "MB_ERR_OOM",
          -5: "MB_ERR_BUDGET", -6: "MB_ERR_HIP", -7: "MB_ERR_NONFINITE", -8: "MB_ERR_STATE",
          -9: "MB_ERR_DEVICE"}
SRC_KIND = {"sech": 0, "gauss": 1, "table": 2}
REC_KIND = {"e": 0, "h": 1, "pop": 2, "inv": 3, "rho_re": 4, "rho_im": 5}
VARIANT = {"auto": 0, "plain": 1, "blocked": 2, "blocked_regs": 3}
FIELD_STEP = {"exact": 0, "cayley": 1}    # MB_FIELD_EXACT, MB_FIELD_CAYLEY

EXPORTS = [
    "mb_last_error", "mb_device_count", "mb_plan_material", "mb_plan_readout", "mb_plan_source", "mb_tile_supported", "mb_workspace_bytes", "mb_setup", "mb_run", "mb_run_static", "mb_run_mode", "mb_batch_run_mode", "mb_reset", "mb_batch_reset", "mb_shape", "mb_batch_shape", "mb_steps_done", "mb_record_shape",
    "mb_read_records", "mb_read_state", "mb_elapsed_ms", "mb_destroy", "mb_batch_setup", "mb_batch_run",
    "mb_batch_record_shape", "mb_batch_read_records", "mb_batch_elapsed_ms", "mb_batch_destroy",
    "mb_server_create", "mb_server_submit", "mb_server_start", "mb_server_drain", "mb_server_cancel", "mb_server_poll",
    "mb_server_status", "mb_server_record_shape", "mb_server_read_records", "mb_server_stats",
    "mb_server_destroy",
]


class MBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class LibraryMissing(RuntimeError):
    pass


# ---------------------------------------------------------------- ABI structs

class mb_qm(C.Structure):
    _fields_ = [("levels", C.c_int32), ("two_level", C.c_int32), ("n3d", C.c_double),
                ("h0_diag", C.POINTER(C.c_double)), ("h0_off", C.POINTER(C.c_double)),
                ("mu_diag", C.POINTER(C.c_double)), ("mu_off", C.POINTER(C.c_double)),
                ("rates", C.POINTER(C.c_double)), ("pure_deph", C.POINTER(C.c_double)),
                ("n_lindblad", C.c_int32), ("lindblad_ops", C.POINTER(C.c_double)),
                ("omega21", C.c_double), ("z21", C.c_double), ("gamma1", C.c_double),
                ("gamma2", C.c_double), ("w0", C.c_double)]


class mb_material(C.Structure):
    _fields_ = [("eps_r", C.c_double), ("mu_r", C.c_double), ("alpha0", C.c_double),
                ("overlap", C.c_double), ("qm", C.POINTER(mb_qm))]


class mb_region(C.Structure):
    _fields_ = [("x_start", C.c_double), ("x_end", C.c_double), ("material", C.c_int32)]


class mb_device_desc(C.Structure):
    _fields_ = [("length", C.c_double), ("refl_left", C.c_double), ("refl_right", C.c_double),
                ("n_materials", C.c_int32), ("materials", C.POINTER(mb_material)),
                ("n_regions", C.c_int32), ("regions", C.POINTER(mb_region))]


class mb_source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("hard", C.c_int32), ("x", C.c_double), ("amp", C.c_double),
                ("freq", C.c_double), ("shift", C.c_double), ("width", C.c_double),
                ("phase", C.c_double), ("period", C.c_double), ("count", C.c_int32),
                ("table", C.POINTER(C.c_double)), ("table_len", C.c_int64)]


class mb_record(C.Structure):
    _fields_ = [("quantity", C.c_int32), ("i", C.c_int32), ("j", C.c_int32), ("cell", C.c_int64),
                ("interval", C.c_int64)]


class mb_consts(C.Structure):
    _fields_ = [("hbar", C.c_double), ("e", C.c_double), ("c0", C.c_double), ("mu0", C.c_double),
                ("eps0", C.c_double)]


class mb_scenario_desc(C.Structure):
    _fields_ = [("nx", C.c_int64), ("dt", C.c_double), ("n_steps", C.c_int64),
                ("precision", C.c_int32), ("variant", C.c_int32), ("block", C.c_int32),
                ("depth", C.c_int32), ("coupling", C.c_int32), ("lanes", C.c_int32),
                ("field_step", C.c_int32),
                ("rho_diag", C.POINTER(C.c_double)),
                ("rho_off", C.POINTER(C.c_double)), ("e_init", C.POINTER(C.c_double)),
                ("n_sources", C.c_int32), ("sources", C.POINTER(mb_source)),
                ("n_records", C.c_int32), ("records", C.POINTER(mb_record)), ("consts", mb_consts),
                ("e_const", C.c_double), ("e_noise", C.c_double), ("e_seed", C.c_uint64)]


_lib = None


def load():
    """Loads libmbhip.so (raises LibraryMissing when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} not built: run paper_2005_05412_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    i64p = C.POINTER(C.c_int64)
    dp = C.POINTER(C.c_double)
    sig = {
        "mb_last_error": (C.c_char_p, []),
        "mb_device_count": (C.c_int, []),
        "mb_plan_material": (C.c_int, [C.POINTER(mb_device_desc), C.POINTER(mb_scenario_desc), C.c_int32,
                                       dp, C.c_int64, i64p]),
        "mb_plan_readout": (C.c_int, [C.POINTER(mb_device_desc), C.POINTER(mb_scenario_desc), C.c_int32,
                                      C.c_int32, dp, C.c_int64]),
        "mb_plan_source": (C.c_int, [C.POINTER(mb_device_desc), C.POINTER(mb_scenario_desc), C.c_int32,
                                     i64p, dp, C.c_int64, i64p]),
        "mb_tile_supported": (C.c_int, [C.c_int32] * 4),
        "mb_setup": (C.c_int, [C.c_int, C.POINTER(mb_device_desc), C.POINTER(mb_scenario_desc), P, C.c_size_t,
                               C.POINTER(P)]),
        "mb_workspace_bytes": (C.c_int, [C.POINTER(mb_device_desc), C.POINTER(mb_scenario_desc),
                                         C.POINTER(C.c_size_t)]),
        "mb_run": (C.c_int, [P, C.c_int64, P]),
        "mb_run_static": (C.c_int, [P, C.c_int64, P]),
        "mb_run_mode": (C.c_int, [P, C.c_int64]),
        "mb_batch_run_mode": (C.c_int, [P]),
        "mb_reset": (C.c_int, [P, P]),
        "mb_batch_reset": (C.c_int, [P, P]),
        "mb_shape": (C.c_int, [P] + [C.POINTER(C.c_int32)] * 4),
        "mb_batch_shape": (C.c_int, [P] + [C.POINTER(C.c_int32)] * 4),
        "mb_steps_done": (C.c_int64, [P]),
        "mb_record_shape": (C.c_int, [P, C.c_int, i64p, i64p]),
        "mb_read_records": (C.c_int, [P, C.c_int, dp, C.c_int64, i64p]),
        "mb_read_state": (C.c_int, [P, dp, dp, dp]),
        "mb_elapsed_ms": (C.c_int, [P, dp]),
        "mb_destroy": (C.c_int, [P]),
        "mb_batch_setup": (C.c_int, [C.c_int, C.c_int32, C.POINTER(mb_device_desc),
                                     C.POINTER(mb_scenario_desc), C.POINTER(P)]),
        "mb_batch_run": (C.c_int, [P, P, C.c_int32]),
        "mb_batch_record_shape": (C.c_int, [P, C.c_int32, C.c_int, i64p, i64p]),
        "mb_batch_read_records": (C.c_int, [P, C.c_int32, C.c_int, dp, C.c_int64, i64p]),
        "mb_batch_elapsed_ms": (C.c_int, [P, dp]),
        "mb_batch_destroy": (C.c_int, [P]),
        "mb_server_create": (C.c_int, [C.c_int, C.c_size_t, C.c_int32, C.c_int32, C.c_int32, C.POINTER(P)]),
        "mb_server_submit": (C.c_int, [P, C.POINTER(mb_device_desc), C.POINTER(mb_scenario_desc),
                                       C.c_double, C.POINTER(C.c_uint64)]),
        "mb_server_start": (C.c_int, [P]),
        "mb_server_drain": (C.c_int, [P, C.c_double]),
        "mb_server_cancel": (C.c_int, [P, C.c_uint64]),
        "mb_server_poll": (C.c_int, [P, C.POINTER(C.c_uint64), C.c_int32, C.POINTER(C.c_int32)]),
        "mb_server_status": (C.c_int, [P, C.c_uint64, C.POINTER(C.c_int32), dp, dp, dp]),
        "mb_server_record_shape": (C.c_int, [P, C.c_uint64, C.c_int, i64p, i64p]),
        "mb_server_read_records": (C.c_int, [P, C.c_uint64, C.c_int, dp, C.c_int64, i64p]),
        "mb_server_stats": (C.c_int, [P, dp, dp, i64p]),
        "mb_server_destroy": (C.c_int, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc, allow_warn=True):
    if rc == MB_OK or (allow_warn and rc > 0):
        return rc
    msg = load().mb_last_error().decode(errors="replace")
    raise MBError(rc, msg)


def _dptr(arr):
    return arr.ctypes.data_as(C.POINTER(C.c_double))


def _complex_pairs(v):
    v = np.asarray(v, complex).reshape(-1)
    out = np.empty(2 * len(v))
    out[0::2] = v.real
    out[1::2] = v.imag
    return out


class _Marshal:
    """Keeps the ctypes structs of one problem and the arrays they point to alive."""

    def __init__(self, prob, precision=None, variant="auto", block=0, depth=0, lanes=0):
        keep = []
        self.keep = keep

        def arr(v):
            a = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
            keep.append(a)
            return _dptr(a)

        mats = (mb_material * len(prob["materials"]))()
        qms = []
        for k, m in enumerate(prob["materials"]):
            mats[k].eps_r, mats[k].mu_r = m["eps_r"], m["mu_r"]
            mats[k].alpha0, mats[k].overlap = m["alpha0"], m["overlap"]
            q = m["qm"]
            if q is None:
                mats[k].qm = None
                continue
            s = mb_qm()
            s.n3d = q["n3d"]
            if q["kind"] == "2lvl":
                s.levels, s.two_level = 2, 1
                s.omega21, s.z21, s.gamma1, s.gamma2, s.w0 = (q["omega21"], q["z21"], q["gamma1"],
                                                              q["gamma2"], q["w0"])
            else:
                s.levels, s.two_level = len(q["h0_diag"]), 0
                s.h0_diag = arr(q["h0_diag"])
                s.h0_off = arr(_complex_pairs(q["h0_off"]))
                s.mu_diag = arr(q["mu_diag"])
                s.mu_off = arr(_complex_pairs(q["mu_off"]))
                s.rates = arr(np.asarray(q["rates"], float).reshape(-1))
                s.pure_deph = arr(q["pure_deph"])
                ops = q.get("lindblad_ops")
                if ops is not None and len(ops):
                    flat = np.asarray(ops, complex).reshape(len(ops), -1)
                    s.n_lindblad = len(ops)
                    s.lindblad_ops = arr(_complex_pairs(flat.reshape(-1)))
            qms.append(s)
            mats[k].qm = C.pointer(s)
        keep.extend([mats, qms])
        regs = (mb_region * len(prob["regions"]))()
        for k, r in enumerate(prob["regions"]):
            regs[k].x_start, regs[k].x_end, regs[k].material = r["x_start"], r["x_end"], r["material"]
        keep.append(regs)
        dev = mb_device_desc()
        dev.length = prob["length"]
        dev.refl_left, dev.refl_right = prob["refl"]
        dev.n_materials, dev.materials = len(prob["materials"]), mats
        dev.n_regions, dev.regions = len(prob["regions"]), regs
        srcs = (mb_source * max(1, len(prob["sources"])))()
        for k, s in enumerate(prob["sources"]):
            srcs[k].kind, srcs[k].hard, srcs[k].x = SRC_KIND[s["kind"]], int(s["hard"]), s["x"]
            srcs[k].amp, srcs[k].freq, srcs[k].shift = s["amp"], s["freq"], s["shift"]
            srcs[k].width, srcs[k].phase, srcs[k].period, srcs[k].count = (s["width"], s["phase"],
                                                                          s["period"], s["count"])
            if s["kind"] == "table":
                srcs[k].table = arr(np.asarray(s["table"], float))
                srcs[k].table_len = len(s["table"])
        recs = (mb_record * max(1, len(prob["records"])))()
        for k, r in enumerate(prob["records"]):
            recs[k].quantity, recs[k].i, recs[k].j = REC_KIND[r["quantity"]], r["i"], r["j"]
            recs[k].cell, recs[k].interval = r["cell"], r["interval"]
        keep.extend([srcs, recs])
        sc = mb_scenario_desc()
        sc.nx, sc.dt, sc.n_steps = prob["nx"], prob["dt"], prob["n_steps"]
        sc.precision = prob["precision"] if precision is None else precision
        sc.variant = VARIANT[variant]
        sc.block, sc.depth, sc.lanes = block, depth, lanes
        sc.coupling = 1 if prob.get("coupling", "weak") == "strong" else 0
        fs = prob.get("field_step", "exact")
        if fs not in FIELD_STEP:
            raise ValueError(f"field_step must be one of {sorted(FIELD_STEP)}, not {fs!r}")
        sc.field_step = FIELD_STEP[fs]
        sc.rho_diag = arr(prob["rho_diag"])
        sc.rho_off = arr(_complex_pairs(prob["rho_off"])) if len(prob["rho_off"]) else arr(np.zeros(1))
        sc.e_init = None if prob["e_init"] is None else arr(prob["e_init"])
        # without an array: constant plus seeded noise drawn by the library
        ef = prob.get("e_field") or {}
        sc.e_const, sc.e_noise, sc.e_seed = ef.get("const", 0.0), ef.get("noise", 0.0), ef.get("seed", 0)
        sc.n_sources, sc.sources = len(prob["sources"]), srcs
        sc.n_records, sc.records = len(prob["records"]), recs
        cs = prob["consts"]
        sc.consts = mb_consts(cs["hbar"], cs["e"], cs["c0"], cs["mu0"], cs["eps0"])
        self.dev, self.scen = dev, sc


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)  # torch.cuda.Stream


# doubles of the largest mb_plan_material output (eight levels: M = 63, K = 56)
_PLAN_CAP = 2 * 63 * 63 + 3 * 63 * 56 + 1024


def plan_material(prob, material, precision=None):
    """Host-only FP64 tables of one material (mb_plan_material), as a dict."""
    lib = load()
    m = _Marshal(prob, precision)
    out = np.zeros(_PLAN_CAP)
    n = C.c_int64()
    rc = _check(lib.mb_plan_material(C.byref(m.dev), C.byref(m.scen), material, _dptr(out), out.size,
                                     C.byref(n)))
    lv = _levels(prob)
    M, K = lv * lv - 1, lv * (lv - 1)
    v = out[: n.value]
    d = {"status": rc}
    if n.value == 0:
        return d
    sizes = [("lam", lv), ("vec", 2 * lv * lv), ("kappa", lv - 1), ("p0", 1), ("at", M), ("ah", M * M), ("bh", M),
             ("am", M * M), ("bf", M), ("t0", K), ("tm", K * M), ("sm", M * K), ("as", K), ("bm", M * K),
             ("lvl", lv), ("block", 1)]
    k = 0
    for name, sz in sizes:
        d[name] = v[k:k + sz].copy()
        k += sz
    d["p0"] = float(d["p0"][0])
    d["vec"] = (d["vec"][0::2] + 1j * d["vec"][1::2]).reshape(lv, lv)
    d["ah"] = d["ah"].reshape(M, M)
    d["am"] = d["am"].reshape(M, M)
    d["tm"] = d["tm"].reshape(K, M)
    d["sm"] = d["sm"].reshape(M, K)
    d["bm"] = d["bm"].reshape(M, K)
    d["lvl"] = d["lvl"].astype(int)
    d["block"] = bool(d["block"][0])
    return d


def plan_readout(prob, record_id, material):
    """Host-only readout vector (r0, r) of a density record for one material."""
    lib = load()
    m = _Marshal(prob)
    lv = _levels(prob)
    out = np.zeros(lv * lv + lv * (lv - 1))
    _check(lib.mb_plan_readout(C.byref(m.dev), C.byref(m.scen), record_id, material, _dptr(out), out.size))
    return out


def tile_supported(levels, precision, block, lanes=1):
    """Whether the blocked kernel is built for this tile (mb_tile_supported); host-only."""
    return bool(load().mb_tile_supported(int(levels), int(precision), int(block), int(lanes)))


def plan_source(prob, source_id, n_values=0):
    """Host-only plan of one source (mb_plan_source): (E node, first n_values table values)."""
    lib = load()
    m = _Marshal(prob)
    node, n = C.c_int64(), C.c_int64()
    out = np.zeros(max(1, n_values))
    _check(lib.mb_plan_source(C.byref(m.dev), C.byref(m.scen), source_id, C.byref(node),
                              _dptr(out) if n_values > 0 else None, n_values, C.byref(n)))
    return node.value, out[: n.value].copy()


def plan_status(prob, precision=None, variant="auto", block=0, depth=0, lanes=0):
    """Status of planning a problem on the host: 0, a positive warning, or raises MBError."""
    lib = load()
    m = _Marshal(prob, precision, variant, block, depth, lanes)
    out = np.zeros(_PLAN_CAP)
    n = C.c_int64()
    for k, mat in enumerate(prob["materials"]):
        rc = _check(lib.mb_plan_material(C.byref(m.dev), C.byref(m.scen), k, _dptr(out), out.size, C.byref(n)))
        if rc:
            return rc
    return 0


def workspace_bytes(prob, precision=None, variant="auto"):
    """Device bytes of one simulation (mb_workspace_bytes): the size of a Solver workspace."""
    m = _Marshal(prob, precision, variant, 0, 0, 0)
    n = C.c_size_t()
    _check(load().mb_workspace_bytes(C.byref(m.dev), C.byref(m.scen), C.byref(n)))
    return n.value


def _workspace_ptr(ws):
    if ws is None:
        return None, 0
    if isinstance(ws, tuple):
        return C.c_void_p(int(ws[0])), int(ws[1])
    return C.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size()


class Solver:
    """One simulation resident on the GPU (mb_setup / mb_run / mb_read_records)."""

    def __init__(self, prob, device=0, precision=None, variant="auto", block=0, depth=0, lanes=0,
                 workspace=None):
        """workspace: None (the library allocates), or caller-owned device memory for the
        simulation, allocated through the same HIP runtime as the library: (pointer, bytes)
        or an object with data_ptr()/numel()/element_size() (kept referenced by the solver),
        at least workspace_bytes(...) bytes, 256-byte aligned."""
        lib = load()
        self.prob = prob
        self._m = _Marshal(prob, precision, variant, block, depth, lanes)
        self._ws = workspace
        ptr, nbytes = _workspace_ptr(workspace)
        h = C.c_void_p()
        self.warning = _check(lib.mb_setup(device, C.byref(self._m.dev), C.byref(self._m.scen), ptr, nbytes,
                                           C.byref(h)))
        self._h = h

    def run(self, n_steps=-1, stream=None):
        _check(load().mb_run(self._h, int(n_steps), _stream_ptr(stream)))
        return self

    def run_static(self, n_steps=-1, stream=None):
        """run() through mb_run_static: no device allocation (tables in the library's static scratch)."""
        _check(load().mb_run_static(self._h, int(n_steps), _stream_ptr(stream)))
        return self

    def reset(self, stream=None):
        _check(load().mb_reset(self._h, _stream_ptr(stream)))
        return self

    def shape(self):
        """(cells per tile, steps per launch, coefficients in registers, waves per 64 cells)."""
        b, d, r, n = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(load().mb_shape(self._h, C.byref(b), C.byref(d), C.byref(r), C.byref(n)))
        return b.value, d.value, bool(r.value), n.value

    def persistent(self, n_steps=None):
        """Whether run(n_steps) (default: all steps) runs its full chunks as persistent launches."""
        n = self.prob["n_steps"] if n_steps is None else int(n_steps)
        r = load().mb_run_mode(self._h, n)
        _check(min(r, 0))
        return r != 0

    @property
    def steps_done(self):
        return int(load().mb_steps_done(self._h))

    def record(self, k):
        lib = load()
        ns, w = C.c_int64(), C.c_int64()
        _check(lib.mb_record_shape(self._h, k, C.byref(ns), C.byref(w)))
        out = np.zeros(max(1, ns.value * w.value))
        n = C.c_int64()
        _check(lib.mb_read_records(self._h, k, _dptr(out), out.size, C.byref(n)))
        out = out[: n.value]
        return out.reshape(ns.value, w.value) if self.prob["records"][k]["cell"] < 0 else out

    def records(self):
        return {r["name"]: self.record(k) for k, r in enumerate(self.prob["records"])}

    def state(self, levels=None):
        nx = self.prob["nx"]
        n = levels if levels is not None else _levels(self.prob)
        e, h = np.zeros(nx), np.zeros(nx)
        rho = np.zeros(nx * max(n, 1) * max(n, 1) * 2)
        _check(load().mb_read_state(self._h, _dptr(e), _dptr(h), _dptr(rho)))
        rho = rho.reshape(nx, max(n, 1), max(n, 1), 2)
        return e, h, rho[..., 0] + 1j * rho[..., 1]

    def elapsed_ms(self):
        ms = C.c_double()
        _check(load().mb_elapsed_ms(self._h, C.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "_h", None):
            load().mb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _levels(prob):
    ns = set()
    for m in prob["materials"]:
        q = m["qm"]
        if q is not None:
            ns.add(2 if q["kind"] == "2lvl" else len(q["h0_diag"]))
    return ns.pop() if ns else 0


class Batch:
    """Many independent simulations advanced together (mb_batch_*)."""

    def __init__(self, probs, device=0, precision=None, variant="auto", block=0, depth=0, lanes=0):
        lib = load()
        self.probs = list(probs)
        self._ms = [_Marshal(p, precision, variant, block, depth, lanes) for p in self.probs]
        n = len(self.probs)
        devs = (mb_device_desc * n)(*[m.dev for m in self._ms])
        scens = (mb_scenario_desc * n)(*[m.scen for m in self._ms])
        self._keep = (devs, scens)
        h = C.c_void_p()
        _check(lib.mb_batch_setup(device, n, devs, scens, C.byref(h)))
        self._h = h

    def run(self, stream=None, use_graph=True):
        _check(load().mb_batch_run(self._h, _stream_ptr(stream), int(bool(use_graph))))
        return self

    def reset(self, stream=None):
        _check(load().mb_batch_reset(self._h, _stream_ptr(stream)))
        return self

    def shape(self):
        """(cells per tile, steps per launch, coefficients in registers, waves per 64 cells)."""
        b, d, r, n = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(load().mb_batch_shape(self._h, C.byref(b), C.byref(d), C.byref(r), C.byref(n)))
        return b.value, d.value, bool(r.value), n.value

    def run_mode(self):
        """How run() advances the full chunks: "flags" (one persistent launch, every tile
        resident), "queue" (work-queue persistent launch), or "chunks" (a launch per chunk)."""
        r = load().mb_batch_run_mode(self._h)
        _check(min(r, 0))
        return {0: "chunks", 1: "flags", 2: "queue"}[r]

    def record(self, sim, k):
        lib = load()
        ns, w = C.c_int64(), C.c_int64()
        _check(lib.mb_batch_record_shape(self._h, sim, k, C.byref(ns), C.byref(w)))
        out = np.zeros(max(1, ns.value * w.value))
        n = C.c_int64()
        _check(lib.mb_batch_read_records(self._h, sim, k, _dptr(out), out.size, C.byref(n)))
        out = out[: n.value]
        return out.reshape(ns.value, w.value) if self.probs[sim]["records"][k]["cell"] < 0 else out

    def records(self, sim):
        return {r["name"]: self.record(sim, k) for k, r in enumerate(self.probs[sim]["records"])}

    def elapsed_ms(self):
        ms = C.c_double()
        _check(load().mb_batch_elapsed_ms(self._h, C.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "_h", None):
            load().mb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching solve server (mb_server_*)."""

    def __init__(self, device=0, hbm_budget=8 << 30, max_slots=256, precision=32, chunk_steps=32):
        lib = load()
        h = C.c_void_p()
        _check(lib.mb_server_create(device, int(hbm_budget), int(max_slots), int(precision),
                                    int(chunk_steps), C.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, prob, arrival_s=0.0):
        m = _Marshal(prob)
        t = C.c_uint64()
        _check(load().mb_server_submit(self._h, C.byref(m.dev), C.byref(m.scen), float(arrival_s), C.byref(t)))
        self._keep[t.value] = [r["cell"] for r in prob["records"]]
        return t.value

    def start(self):
        _check(load().mb_server_start(self._h))

    def drain(self, timeout_s=600.0):
        _check(load().mb_server_drain(self._h, float(timeout_s)))

    def cancel(self, ticket):
        _check(load().mb_server_cancel(self._h, C.c_uint64(ticket)))

    def poll(self, capacity=256):
        """Tickets that reached a final state since the previous poll (non-blocking)."""
        buf = (C.c_uint64 * max(1, capacity))()
        n = C.c_int32()
        _check(load().mb_server_poll(self._h, buf, int(capacity), C.byref(n)))
        return [int(buf[i]) for i in range(n.value)]

    def status(self, ticket):
        st, ta, tb, tc = C.c_int32(), C.c_double(), C.c_double(), C.c_double()
        _check(load().mb_server_status(self._h, C.c_uint64(ticket), C.byref(st), C.byref(ta), C.byref(tb),
                                       C.byref(tc)))
        return st.value, ta.value, tb.value, tc.value

    def record(self, ticket, k):
        lib = load()
        ns, w = C.c_int64(), C.c_int64()
        _check(lib.mb_server_record_shape(self._h, C.c_uint64(ticket), k, C.byref(ns), C.byref(w)))
        out = np.zeros(max(1, ns.value * w.value))
        n = C.c_int64()
        _check(lib.mb_server_read_records(self._h, C.c_uint64(ticket), k, _dptr(out), out.size, C.byref(n)))
        out = out[: n.value]
        return out.reshape(ns.value, w.value) if self._keep[ticket][k] < 0 else out

    def stats(self):
        cu, busy, ch = C.c_double(), C.c_double(), C.c_int64()
        _check(load().mb_server_stats(self._h, C.byref(cu), C.byref(busy), C.byref(ch)))
        return cu.value, busy.value, ch.value

    def close(self):
        if getattr(self, "_h", None):
            load().mb_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
