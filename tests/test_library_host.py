"""Host-side checks of libmbhip.so that need no GPU.

* the shared library loads and exports every function ``include/mb.h`` declares;
* the library's own FP64 plan (Jacobi eigen-basis of mu, real trace-eliminated
  Liouvillian, Taylor scaling-and-squaring exponentials, polarization and
  record readouts) reproduces the oracle's single-point solve when its tables
  are stepped in the kernels' formulation (rotation by E, p = at.y + p0,
  sigma' = y + am y + bf);
* invalid descriptions map to the documented status codes.
"""
import math
import os
import re

import numpy as np
import pytest

import paper_2005_05412_amd as mb
import workloads as W
from oracle import mb_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
C = W.CODATA


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mb_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = mb.load()
    names = declared_functions()
    assert len(names) >= 28
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(mb.EXPORTS) == names


def test_no_gpu_means_no_device_here():
    # the container has no GPU; the call must still return cleanly
    assert mb.load().mb_device_count() >= 0


# ---------------------------------------------------------------- plan tables vs oracle

def _rho_to_x(rho_p, n):
    x = [rho_p[k, k].real for k in range(n - 1)]
    for j in range(1, n):
        for i in range(j):
            x += [rho_p[i, j].real, rho_p[i, j].imag]
    return np.array(x)


def _x_to_rho(x, n):
    r = np.zeros((n, n), complex)
    for k in range(n - 1):
        r[k, k] = x[k]
    r[n - 1, n - 1] = 1.0 - sum(x[: n - 1])
    q = 0
    for j in range(1, n):
        for i in range(j):
            z = x[n - 1 + 2 * q] + 1j * x[n + 2 * q]
            r[i, j], r[j, i] = z, np.conj(z)
            q += 1
    return r


def _increments(z, e, kappa, n):
    """(e^{i theta_jk} - 1) z_jk for the eigenbasis pairs j < k, theta_jk = e sum kappa[j:k]."""
    d = np.zeros_like(z)
    q = 0
    for k in range(1, n):
        for j in range(k):
            th = e * sum(kappa[j:k])
            w = (z[2 * q] + 1j * z[2 * q + 1]) * (np.exp(1j * th) - 1.0)
            d[2 * q], d[2 * q + 1] = w.real, w.imag
            q += 1
    return d


def _random_ops(rng, n, k=3, rate=1e12):
    """k random complex N x N Lindblad operators of size ~ sqrt(rate)."""
    return [(rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) * np.sqrt(rate / n) for _ in range(k)]


@pytest.mark.parametrize("n,seed,ops", [(2, 1, False), (3, 2, False), (4, 3, False), (5, 4, False), (6, 5, False),
                                        (7, 8, False), (8, 9, False), (3, 6, True), (5, 7, True)])
def test_plan_tables_reproduce_oracle_single_point(n, seed, ops):
    rng = np.random.default_rng(seed)
    qm = W.random_qm(rng, n, dipole=3e-29)
    if ops:                                  # explicit Lindblad operators replace the rates
        qm["lindblad_ops"] = _random_ops(rng, n)
    rd, ro = W.random_rho(rng, n)
    src = W.source("sech", 0, 3e9, 2e14, 5.0, 1.0 / 15e-15, phase=0.4)
    dt, nt = 2e-17, 600
    prob = W.make_problem("pt", 0.0, [W.qm_material(qm)], [(0.0, 0.0, 0)], 1, dt, nt, rd, ro,
                          sources=[src], records=[])
    t = mb.plan_material(prob, 0)
    orc = O.Oracle(prob)
    V = t["vec"]
    lvl = t["lvl"]
    # the tables order the levels so that the most populated initial one is last
    assert lvl[int(np.argmax(rd))] == n - 1 and sorted(lvl) == list(range(n))
    order = np.argsort(lvl)                  # internal level k is the caller's level order[k]
    rho0 = O.unpack_hermitian(rd, ro)
    sigma = t["ah"] @ _rho_to_x(rho0[np.ix_(order, order)], n) + t["bh"]
    # eigen-decomposition of mu is the library's own
    mu = O.describe(qm, C)[1][np.ix_(order, order)]
    assert np.allclose(V @ np.diag(t["lam"]) @ V.conj().T, mu, rtol=0, atol=1e-12 * abs(mu).max())
    errs = []
    for step in range(nt):
        e = orc.e[0]
        z = t["t0"] + t["tm"] @ sigma
        # z holds the coherences of V^+ rho V
        if step == 0:
            rs = V.conj().T @ _x_to_rho(sigma, n) @ V
            zz = np.array([[rs[j, k].real, rs[j, k].imag] for k in range(1, n) for j in range(k)]).ravel()
            assert np.allclose(z, zz, rtol=0, atol=1e-13)
        d = _increments(z, e, t["kappa"], n)
        y = sigma + t["sm"] @ d
        p = t["at"] @ y + t["p0"]
        assert abs(p - (t["at"] @ sigma + t["as"] @ d + t["p0"])) <= 1e-12 * max(1.0, abs(p))
        rho_half = _x_to_rho(t["ah"] @ y + t["bh"], n)[np.ix_(lvl, lvl)]
        new = sigma + t["am"] @ sigma + t["bm"] @ d + t["bf"]
        sigma = y + t["am"] @ y + t["bf"]
        assert np.max(np.abs(new - sigma)) < 1e-13
        orc.step()
        ref = orc.full_density()[0]
        errs.append(np.max(np.abs(rho_half - ref)))
        assert abs(p - orc.p_cur[0]) <= 1e-9 * max(1.0, abs(orc.p_cur[0])) + 1e-12 * np.abs(orc.p_cur).max()
    assert max(errs) < 1e-12


def test_plan_readouts_match_oracle_quantities():
    rng = np.random.default_rng(7)
    n = 4
    qm = W.random_qm(rng, n)
    rd, ro = W.random_rho(rng, n)
    recs = [W.record("p2", "pop", 0, 1, 2, 2), W.record("inv", "inv", 0, 1, 1, 3),
            W.record("re", "rho_re", 0, 1, 0, 2), W.record("im", "rho_im", 0, 1, 1, 3)]
    prob = W.make_problem("pt", 0.0, [W.qm_material(qm)], [(0.0, 0.0, 0)], 1, 2e-17, 5, rd, ro,
                          e_init=np.array([2e9]), records=recs)
    t = mb.plan_material(prob, 0)
    orc = O.Oracle(prob)
    M = n * n - 1
    order = np.argsort(t["lvl"])
    sigma = t["ah"] @ _rho_to_x(O.unpack_hermitian(rd, ro)[np.ix_(order, order)], n) + t["bh"]
    d = _increments(t["t0"] + t["tm"] @ sigma, 2e9, t["kappa"], n)
    r = orc.run(1)
    for k, rec in enumerate(recs):
        ro_vec = mb.plan_readout(prob, k, 0)
        assert ro_vec.size == M + 1 + n * (n - 1)
        val = ro_vec[0] + ro_vec[1:1 + M] @ sigma + ro_vec[1 + M:] @ d
        assert abs(val - r[rec["name"]][0]) < 1e-13


def test_two_level_constructor_matches_oracle():
    qm = W.two_level_params(1e24, 2 * math.pi * 2e14, 6.24e-11, 1e10, 3e10, -0.5)
    prob = W.make_problem("pt", 0.0, [W.qm_material(qm)], [(0.0, 0.0, 0)], 1, 1e-17, 3, [1.0, 0.0],
                          records=[])
    t = mb.plan_material(prob, 0)
    h0, mu, rates, deph, _ = O.describe(qm, C)
    assert np.allclose(np.sort(t["lam"]), np.linalg.eigvalsh(mu), rtol=1e-14)


# ---------------------------------------------------------------- status codes

def _vac(nx=20, courant=0.5, refl=(0.0, 0.0), levels_qm=None):
    L = 1e-5
    mats = [W.vacuum()] if levels_qm is None else [W.qm_material(levels_qm)]
    dt = W.courant_dt(L, nx, C["c0"], courant)
    rho = [1.0] if levels_qm is None else [1.0] + [0.0] * (W.qm_levels(levels_qm) - 1)
    return W.make_problem("v", L, mats, [(0.0, L, 0)], nx, dt, 10, rho, refl=refl)


def test_status_codes():
    assert mb.plan_status(_vac()) == 0
    with pytest.raises(mb.MBError) as ex:    # two nodes: edges only, no interior to update
        mb.plan_status(_vac(nx=2))
    assert ex.value.code == -1
    with pytest.raises(mb.MBError) as ex:
        mb.plan_status(_vac(courant=1.01))
    assert ex.value.code == -2
    assert mb.plan_status(_vac(refl=(0.5, 0.8))) == 0      # semi-transparent ends
    for bad_r in ((1.5, 0.0), (0.0, -0.1)):
        with pytest.raises(mb.MBError) as ex:
            mb.plan_status(_vac(refl=bad_r))
        assert ex.value.code == -1
    rng = np.random.default_rng(1)
    assert mb.plan_status(_vac(levels_qm=W.random_qm(rng, 8))) == 0
    with pytest.raises(mb.MBError) as ex:
        mb.plan_status(_vac(levels_qm=W.random_qm(rng, 9)))
    assert ex.value.code == -3
    for key, val in (("coupling", "strong"), ("field_step", "cayley")):
        big = _vac(levels_qm=W.random_qm(rng, 7))   # 7 and 8 levels: weak coupling, exact field step
        big[key] = val
        with pytest.raises(mb.MBError) as ex:
            mb.plan_status(big)
        assert ex.value.code == -3
    bad = _vac()
    bad["regions"] = [dict(x_start=0.0, x_end=0.5e-5, material=0)]
    with pytest.raises(mb.MBError) as ex:
        mb.plan_status(bad)
    assert ex.value.code == -1
    for x in (1e-5 * (1 + 0.6 / 19), -0.6e-5 / 19, float("nan")):     # beyond either end by > dx/2
        bad = _vac()
        bad["sources"] = [W.source("sech", x, 1.0, 1e14, 1.0, 1e14)]
        with pytest.raises(mb.MBError) as ex:
            mb.plan_status(bad)
        assert ex.value.code == -1
    bad = _vac()
    bad["sources"] = [W.table_source(W.node_x(1e-5, 20, 3), [0.0, np.nan, 1.0])]
    with pytest.raises(mb.MBError) as ex:
        mb.plan_status(bad)
    assert ex.value.code == -1
    ok = _vac()
    ok["sources"] = [W.table_source(W.node_x(1e-5, 20, 3), [0.0, 0.5, 1.0]),
                     W.table_source(W.node_x(1e-5, 20, 4), [], hard=False)]
    assert mb.plan_status(ok) == 0
    # waves per 64 cells: 0 (default), 1, 2, 4 or 8
    for lanes in (0, 1, 2, 4, 8):
        assert mb.plan_status(_vac(), lanes=lanes) == 0
    for lanes in (3, 16, -1):
        with pytest.raises(mb.MBError) as ex:
            mb.plan_status(_vac(), lanes=lanes)
        assert ex.value.code == -1
    with pytest.raises(mb.MBError) as ex:
        mb.plan_status(_vac(), precision=32, variant="plain")
    assert ex.value.code == -3
    strong = _vac()
    strong["coupling"] = "strong"
    assert mb.plan_status(strong) == 0
    with pytest.raises(mb.MBError) as ex:        # strong coupling runs on the blocked variant
        mb.plan_status(strong, variant="plain")
    assert ex.value.code == -3
    cay = _vac()
    cay["field_step"] = "cayley"
    assert mb.plan_status(cay) == 0
    assert mb.plan_status(cay, variant="plain") == 0
    assert mb.plan_status(cay, variant="blocked_regs") == 0
    cay["field_step"] = "pade"
    with pytest.raises(ValueError):
        mb.plan_status(cay)


def test_workspace_bytes():
    """mb_workspace_bytes: host-only, 256-byte granules, at least the two state copies of
    E, H and the M density planes, growing with the grid and the precision."""
    p = W.random_small(12, N=3, nx=150, n_steps=90)
    b64 = mb.workspace_bytes(p, precision=64)
    b32 = mb.workspace_bytes(p, precision=32)
    assert b64 % 256 == 0 and b32 % 256 == 0
    m = 8
    assert b64 >= 2 * (2 + m) * 150 * 8 and b32 >= 2 * (2 + m) * 150 * 4
    assert b32 < b64
    big = W.random_small(12, N=3, nx=1500, n_steps=90)
    assert mb.workspace_bytes(big, precision=64) > b64
    with pytest.raises(mb.MBError) as ex:
        mb.workspace_bytes(_vac(courant=1.01))
    assert ex.value.code == -2


def test_non_completely_positive_dephasing_warns():
    qm = W.general_qm(1e24, [0.0, 0.1 * C["e"], 0.2 * C["e"]], None, None,
                      np.array([1e-29, 1e-29, 0.0]), np.zeros((3, 3)), [1e12, 1e12, 10e12])
    assert mb.plan_status(_vac(levels_qm=qm)) == mb.MB_WARN_NOT_CP
    ok = W.general_qm(1e24, [0.0, 0.1 * C["e"], 0.2 * C["e"]], None, None,
                      np.array([1e-29, 1e-29, 0.0]), np.zeros((3, 3)), [1e12, 1e12, 1e12])
    assert mb.plan_status(_vac(levels_qm=ok)) == 0


def test_splitmix64_published_outputs():
    """The seeded generator the inputs are drawn from is SplitMix64: for seed 0 its first
    outputs are 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f (the published
    reference sequence), mapped to [0, 1) by their top 53 bits."""
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    got = W.splitmix64_uniform(0, 3)
    assert list(got) == [(z >> 11) * 2.0 ** -53 for z in want]


def test_source_positions_convert_like_the_oracle():
    """The library puts a source at the node the oracle does: round(x/dx), halves to the
    even node (Sec. 3.2 converts positions to grid indices), and its FP64 value table is
    the oracle's source at t_n = n dt."""
    prob = _vac(nx=21)
    dx = prob["length"] / 20
    xs = [0.0, 0.3 * dx, 0.5 * dx, 1.5 * dx, 2.5 * dx, 7.49 * dx, 7.5 * dx, 19.5 * dx, prob["length"],
          prob["length"] + 0.4 * dx]
    prob["sources"] = [W.source("gauss", x, 2e8, 1.9e14, 3.0, 1.0 / 5e-15, phase=0.3) for x in xs]
    orc = O.Oracle(prob)
    for k, x in enumerate(xs):
        node, vals = mb.plan_source(prob, k, n_values=prob["n_steps"] + 1)
        assert node == O.source_cell(x, dx, 21) == orc.src_cell[k], (k, x / dx)
        want = [O.source_value(prob["sources"][k], n * prob["dt"]) for n in range(prob["n_steps"] + 1)]
        assert np.max(np.abs(vals - want)) <= 1e-15 * 2e8
    assert [orc.src_cell[k] for k in range(len(xs))] == [0, 0, 0, 2, 2, 7, 8, 20, 20, 20]
