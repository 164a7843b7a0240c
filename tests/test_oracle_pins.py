"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's
own formula: they use closed forms, an independent ODE form (the optical
Bloch equations of Sec. 3.1.1), an independent Kronecker-product construction
of the Liouvillian, conservation laws and the paper's printed numbers.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.integrate import solve_ivp

import workloads as W
from oracle import mb_oracle as O

C = W.CODATA
HB = C["hbar"]


def single_point(qm, n_steps, dt, rho_diag, rho_off=None, e_const=0.0, sources=(), records=None):
    """Nx = 1 problem: the pure Lindblad solve of Sec. 3.2 / Sec. 4.2."""
    n = W.qm_levels(qm)
    if records is None:
        records = [W.record(f"p{i}", "pop", 0, 1, i=i, j=i) for i in range(n)]
        records += [W.record(f"re{i}{j}", "rho_re", 0, 1, i=i, j=j) for (i, j) in O.pair_list(n)]
        records += [W.record(f"im{i}{j}", "rho_im", 0, 1, i=i, j=j) for (i, j) in O.pair_list(n)]
    e_init = None if e_const == 0.0 else np.array([e_const])
    return W.make_problem("pt", 0.0, [W.qm_material(qm)], [(0.0, 0.0, 0)], 1, dt, n_steps,
                          rho_diag, rho_off, e_init=e_init, sources=list(sources), records=records)


def two_level(omega21, z21, gamma1, gamma2, w0, n3d=1e24):
    return W.two_level_params(n3d, omega21, z21, gamma1, gamma2, w0)


# ---------------------------------------------------------------- P1 relaxation

def test_p1_two_level_relaxation_closed_form():
    """E = 0: w(t) = w0 + (w(0) - w0) e^{-gamma1 t}; rho21 = rho21(0) e^{-(i w21 + gamma2) t}
    (optical Bloch equations, Sec. 3.1.1)."""
    om, g1, g2, w0 = 2 * math.pi * 1e13, 3e11, 7e11, 0.2
    qm = two_level(om, 1e-10, g1, g2, w0)
    dt, nt = 1e-15, 4000
    rho_d, rho_o = [0.3, 0.7], [0.2 + 0.1j]          # rho_12 = 0.2 + 0.1 i
    recs = O.Oracle(single_point(qm, nt, dt, rho_d, rho_o)).run()
    t = (np.arange(nt) + 1) * dt                     # rho^{n+1/2} sits at (n+1) dt from rho^{-1/2}
    w = recs["p1"] - recs["p0"]
    w_ref = w0 + (0.4 - w0) * np.exp(-g1 * t)
    assert np.max(np.abs(w - w_ref)) < 1e-12
    r21 = recs["re01"] - 1j * recs["im01"]           # rho_21 = conj(rho_12)
    r21_ref = (0.2 - 0.1j) * np.exp(-(1j * om + g2) * t)
    assert np.max(np.abs(r21 - r21_ref)) < 1e-12


@pytest.mark.parametrize("n", [3, 4, 6])
def test_p1_single_channel_population_transfer(n):
    """Only gamma_ij != 0 and all population in j: rho_ii(t) = 1 - e^{-gamma_ij t}
    (eq:relax_pop with the rate matrix read as gamma_ij = rate j -> i)."""
    rng = np.random.default_rng(n)
    for _ in range(3):
        i, j = rng.choice(n, 2, replace=False)
        rates = np.zeros((n, n))
        rates[i, j] = 5e11
        en = np.sort(rng.uniform(0, 0.3, n)) * C["e"]
        qm = W.general_qm(1e24, en, None, None, None, rates, np.zeros(n * (n - 1) // 2))
        rho = np.zeros(n)
        rho[j] = 1.0
        dt, nt = 2e-15, 1500
        recs = O.Oracle(single_point(qm, nt, dt, rho)).run()
        t = (np.arange(nt) + 1) * dt
        assert np.max(np.abs(recs[f"p{i}"] - (1 - np.exp(-5e11 * t)))) < 1e-12
        assert np.max(np.abs(recs[f"p{j}"] - np.exp(-5e11 * t))) < 1e-12
        others = [k for k in range(n) if k not in (i, j)]
        for k in others:
            assert np.max(np.abs(recs[f"p{k}"])) < 1e-14


# ---------------------------------------------------------------- P2 / P3 Rabi

@pytest.mark.parametrize("n", [2, 3, 5])
def test_field_free_medium_in_a_stationary_state_stays_field_free(n):
    """With no field the field factor is exp(0) = I (Sec. 2.2) and the ground state of a
    ladder that only decays downward is stationary under L0 (eq:relax_pop: nothing leaves
    level 1), so its polarization n3D tr{mu L0(rho)} vanishes (mu has no diagonal) and a
    medium left alone in it radiates nothing: E stays exactly zero everywhere."""
    prob = W.ladder(n, nx=120, n_steps=300, rec_interval=1)
    prob["sources"] = []
    orc = O.Oracle(prob)
    for _ in range(prob["n_steps"]):
        orc.step()
        assert not np.any(orc.e) and not np.any(orc.p_cur)
    rho = orc.groups[0]["rho"]
    assert np.all(rho[:, 0, 0] == 1.0) and np.count_nonzero(rho) == rho.shape[0]


def test_p2_resonant_rabi_exact_when_h0_vanishes():
    """H0 = 0, no relaxation, constant E: the splitting is exact and
    rho_22(t) = sin^2(mu12 E t / hbar)."""
    z21 = 1e-10
    qm = two_level(0.0, z21, 0.0, 0.0, -1.0)
    e_c, dt, nt = 1e8, 5e-16, 3000
    recs = O.Oracle(single_point(qm, nt, dt, [1.0, 0.0], e_const=e_c)).run()
    t = (np.arange(nt) + 1) * dt
    mu12 = C["e"] * z21
    assert np.max(np.abs(recs["p1"] - np.sin(mu12 * e_c * t / HB) ** 2)) < 1e-12


def _rabi_error(dt):
    om, z21 = 2 * math.pi * 1e14, 1e-29 / C["e"]
    mu12 = 1e-29
    e_c = 0.25 * HB * om / mu12
    qm = two_level(om, z21, 0.0, 0.0, -1.0)
    t_end = 2e-13
    nt = int(round(t_end / dt))
    recs = O.Oracle(single_point(qm, nt, dt, [1.0, 0.0], e_const=e_c)).run()
    t = (np.arange(nt) + 1) * dt
    om_c = 2 * mu12 * e_c / HB
    om_p = math.sqrt(om ** 2 + om_c ** 2)
    ref = (om_c / om_p) ** 2 * np.sin(om_p * t / 2) ** 2
    return np.max(np.abs(recs["p1"] - ref))


def test_p3_generalized_rabi_second_order():
    """H0 != 0, constant E: generalized Rabi formula P2 = (Wc/W')^2 sin^2(W' t/2),
    Wc = 2 mu12 E/hbar, W' = sqrt(w21^2 + Wc^2); Strang splitting is second order."""
    errs = [_rabi_error(dt) for dt in (4e-17, 2e-17, 1e-17)]
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert errs[-1] < 1e-4
    for o in orders:
        assert 1.9 < o < 2.1, (errs, orders)


# ---------------------------------------------------------------- P4 optical Bloch equations

def _obe_error(dt):
    """Oracle vs the optical Bloch equations (Sec. 3.1.1) under a sech drive."""
    om, z21, g1, g2, w0 = 2 * math.pi * 1e14, 8e-11, 2e12, 5e12, -0.6
    qm = two_level(om, z21, g1, g2, w0)
    src = W.source("sech", 0, 2e9, 1e14, 6.0, 1.0 / 10e-15, phase=0.3)
    t_end = 160e-15
    nt = int(round(t_end / dt))
    rec = [W.record("p0", "pop", 0, 1, 0, 0), W.record("p1", "pop", 0, 1, 1, 1),
           W.record("re", "rho_re", 0, 1, 0, 1), W.record("im", "rho_im", 0, 1, 0, 1)]
    prob = single_point(qm, nt, dt, [0.8, 0.2], [0.0], sources=[src], records=rec)
    recs = O.Oracle(prob).run()
    mu21 = -C["e"] * z21

    def e_of_t(t):
        return src["amp"] / math.cosh(src["width"] * t - src["shift"]) * math.sin(
            2 * math.pi * src["freq"] * t + src["phase"])

    def rhs(t, y):
        r21 = y[0] + 1j * y[1]
        w = y[2]
        om_r = mu21 * e_of_t(t) / HB
        dr = -1j * om * r21 - 1j * w * om_r - g2 * r21
        dw = 4 * om_r * r21.imag - g1 * (w - w0)
        return [dr.real, dr.imag, dw]

    # rho^{-1/2} = rho_init at t = -dt/2 (weak coupling, Fig. 1)
    sol = solve_ivp(rhs, (-dt / 2, t_end), [0.0, 0.0, -0.6], method="DOP853",
                    rtol=1e-12, atol=1e-14, dense_output=True)
    t = (np.arange(nt) + 1) * dt - dt / 2
    y = sol.sol(t)
    w = recs["p1"] - recs["p0"]
    r21 = recs["re"] - 1j * recs["im"]
    return max(np.max(np.abs(w - y[2])), np.max(np.abs(r21 - (y[0] + 1j * y[1]))))


def test_p4_optical_bloch_equations_second_order():
    errs = [_obe_error(dt) for dt in (4e-17, 2e-17, 1e-17)]
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert errs[-1] < 1e-4
    for o in orders:
        assert 1.85 < o < 2.15, (errs, orders)


# ---------------------------------------------------------------- P5 local error vs brute force

def _kron_liouvillian(h, mu, e, ops):
    """Independent superoperator: row-major vec(A X B) = (A kron B^T) vec(X)."""
    n = h.shape[0]
    eye = np.eye(n)
    hf = h - mu * e
    lv = -1j / HB * (np.kron(hf, eye) - np.kron(eye, hf.T))
    for op in ops:
        ld = op.conj().T
        lv += np.kron(op, op.conj()) - 0.5 * (np.kron(ld @ op, eye) + np.kron(eye, (ld @ op).T))
    return lv


@pytest.mark.parametrize("n", [2, 3, 5])
def test_p5_one_step_local_error_third_order(n):
    """One Strang step vs expm((L0 + L_E) dt): local error O(dt^3)."""
    rng = np.random.default_rng(10 + n)
    qm = W.random_qm(rng, n, dipole=3e-29)
    h0, mu, rates, deph, _ = O.describe(qm, C)
    ops, lam_min = O.lindblad_from_rates(rates, deph)
    assert lam_min >= -1e-9 * deph.max()
    rd, ro = W.random_rho(rng, n)
    rho0 = O.unpack_hermitian(rd, ro)
    e = 3e9
    errs = []
    for dt in (2e-17, 1e-17, 5e-18):
        prob = single_point(qm, 1, dt, rd, ro, e_const=e, records=[])
        orc = O.Oracle(prob)
        orc.step()
        got = orc.full_density()[0]
        lv = _kron_liouvillian(h0, mu, e, ops)
        ref = (sla.expm(lv * dt) @ rho0.reshape(-1)).reshape(n, n)
        errs.append(np.max(np.abs(got - ref)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 6.5 < r1 < 9.5 and 6.5 < r2 < 9.5, errs


# ---------------------------------------------------------------- P6 invariants

@pytest.mark.parametrize("n,seed", [(2, 1), (3, 2), (4, 3), (6, 4)])
def test_p6_density_invariants(n, seed):
    """Trace one, Hermitian, positive semi-definite in every quantum cell (Sec. 2.2)."""
    prob = W.random_small(seed, N=n, nx=30, n_steps=80, full_records=False)
    orc = O.Oracle(prob)
    for _ in range(80):
        orc.step()
        for g in orc.groups:
            rho = g["rho"]
            tr = np.trace(rho, axis1=1, axis2=2)
            assert np.max(np.abs(tr - 1.0)) < 1e-12
            assert np.max(np.abs(rho - np.conj(np.transpose(rho, (0, 2, 1))))) < 1e-14
            lam = np.linalg.eigvalsh(rho)
            assert lam.min() > -1e-12


# ---------------------------------------------------------------- P7 FDTD energy, CFL

def _vacuum_problem(nx, courant, n_steps, refl=(1.0, 1.0), e_init=None, records=(), mats=None,
                    regions=None, sources=()):
    L = 1e-4
    mats = mats or [W.vacuum()]
    regions = regions or [(0.0, L, 0)]
    c_max = max(O.light_speed(m, C) for m in mats)
    dt = W.courant_dt(L, nx, c_max, courant)
    return W.make_problem("vac", L, mats, regions, nx, dt, n_steps, [1.0], refl=refl,
                          e_init=e_init, records=list(records), sources=list(sources))


def test_p7_discrete_energy_conserved_in_lossless_vacuum():
    """Yee scheme, sigma = 0, PEC ends: W^n = sum eps E^2 dx/2 + sum mu H^{n+1/2} H^{n-1/2} dx/2
    is invariant for c dt <= dx."""
    nx, nt = 400, 20000
    x = np.arange(nx)
    e0 = np.exp(-((x - 150) / 12.0) ** 2) * np.sin(x / 3.0) * 1e6
    e0[0] = e0[-1] = 0.0
    prob = _vacuum_problem(nx, 0.5, nt, e_init=e0,
                           records=[W.record("e", "e", -1, 1), W.record("h", "h", -1, 1)])
    recs = O.Oracle(prob).run()
    dx = prob["length"] / (nx - 1)
    eps, mu = C["eps0"], C["mu0"]
    e, h = recs["e"], recs["h"][:, :-1]             # e[k] = E^{k+1}, h[k] = H^{k+1/2}
    w = 0.5 * eps * dx * np.sum(e[:-1] ** 2, axis=1) + 0.5 * mu * dx * np.sum(h[1:] * h[:-1], axis=1)
    assert np.max(np.abs(w / w[0] - 1.0)) < 1e-12


def test_p7_courant_limit_guard():
    with pytest.raises(ValueError):
        O.Oracle(_vacuum_problem(50, 1.01, 10))


def test_p7_magic_time_step_shifts_one_cell():
    """C = 1 in vacuum: a right-moving wave moves exactly one cell per step."""
    nx = 300
    x = np.arange(nx)
    prob = _vacuum_problem(nx, 1.0, 100, refl=(0.0, 0.0),
                           records=[W.record("e", "e", -1, 1)])
    # launch a right-going wave with a soft line of sources: use the initial field and
    # an initial H consistent with a right-moving pulse (H^{-1/2} from E at x - c dt/2)
    orc = O.Oracle(prob)
    f = lambda s: np.exp(-((s - 80.0) / 6.0) ** 2)
    orc.e[:] = f(x)
    eta = math.sqrt(C["mu0"] / C["eps0"])
    orc.h[:] = -f(x[:-1] + 0.5 + 0.5) / eta          # H^{-1/2} at x_{m+1/2}, t = -dt/2
    recs = orc.run()
    for n in (20, 60, 99):
        assert np.max(np.abs(recs["e"][n - 1] - f(x - n))) < 1e-12


def test_p7_table_source_is_translated_one_cell_per_step():
    """A hard sampled-waveform source (table[n] at t_n = n dt) at cell 0 of a vacuum grid
    at C = 1: the discrete wave equation is exact there, so E_m^n = table[n - m] (zero
    outside the table)."""
    rng = np.random.default_rng(3)
    vals = rng.normal(size=40)
    nx, steps = 120, 70
    prob = _vacuum_problem(nx, 1.0, steps, refl=(0.0, 0.0), records=[W.record("e", "e", -1, 1)],
                           sources=[W.table_source(0, vals)])
    recs = O.run(prob)
    for n in (1, 25, 39, 55, 70):
        want = np.array([vals[n - m] if 0 <= n - m < len(vals) else 0.0 for m in range(nx)])
        assert np.max(np.abs(recs["e"][n - 1] - want)) < 1e-12, n
    # a table holding an analytic waveform's samples gives that waveform's run exactly
    src = W.source("gauss", 0, 1.0, 3e13, 4.0, 1.0 / 20e-15)
    p1 = _vacuum_problem(nx, 0.9, steps, refl=(0.0, 0.0), records=[W.record("e", "e", -1, 1)], sources=[src])
    samples = [O.source_value(src, n * p1["dt"]) for n in range(steps + 1)]
    p2 = _vacuum_problem(nx, 0.9, steps, refl=(0.0, 0.0), records=[W.record("e", "e", -1, 1)],
                         sources=[W.table_source(0, samples)])
    assert np.array_equal(O.run(p1)["e"], O.run(p2)["e"])


# ---------------------------------------------------------------- P8 loss

def test_p8_lossy_background_field_decay():
    """alpha0 = sqrt(mu/eps) sigma/2 is the field attenuation (Sec. 3.1.1): a CW wave
    in a low-loss medium decays as e^{-alpha0 x}."""
    alpha0, lam = 2e4, 1.5e-6
    nx = 2001
    L = lam / 100 * (nx - 1)                          # dx = lam / 100
    mat = W.vacuum(eps_r=1.0, alpha0=alpha0)
    dt = W.courant_dt(L, nx, C["c0"], 0.5)
    f = C["c0"] / lam
    src = W.source("sech", 0, 1.0, f, 0.0, 1e6)       # sech(1e6 t) ~ 1: continuous wave
    c1, c2 = 400, 1400
    nt = 12000
    prob = W.make_problem("loss", L, [mat], [(0.0, L, 0)], nx, dt, nt, [1.0], refl=(0.0, 0.0),
                          sources=[src], records=[W.record("a", "e", c1, 1), W.record("b", "e", c2, 1)])
    recs = O.Oracle(prob).run()
    tail = slice(nt - 2000, nt)
    amp1 = np.max(np.abs(recs["a"][tail]))
    amp2 = np.max(np.abs(recs["b"][tail]))
    dx = L / (nx - 1)
    ref = math.exp(-alpha0 * (c2 - c1) * dx)
    assert abs(amp2 / amp1 / ref - 1.0) < 2e-3


# ---------------------------------------------------------------- boundary conditions

def test_absorbing_and_reflecting_ends():
    """R = 0 absorbs an outgoing pulse (first-order Mur); R = 1 reflects it with E -> -E."""
    nx = 400
    x = np.arange(nx)
    e0 = np.exp(-((x - 200) / 10.0) ** 2) * 1e6
    for refl in ((0.0, 0.0), (1.0, 1.0)):
        prob = _vacuum_problem(nx, 0.5, 800, refl=refl, e_init=e0,
                               records=[W.record("e", "e", -1, 1)])
        recs = O.Oracle(prob).run()
        e = recs["e"]
        w0 = np.sum(e0 ** 2)
        w_end = np.sum(e[-1] ** 2)
        if refl[0] == 0.0:
            assert w_end / w0 < 1e-4
        else:
            # the two halves travel 400 cells: each hits its wall once and they meet
            # again near the start with the sign flipped
            assert e[-1][199] < -0.8 * 1e6


@pytest.mark.parametrize("refl", [0.25, 0.64, 0.9])
def test_semi_transparent_end_reflects_r_equal_minus_sqrt_R(refl):
    """0 < R < 1 (semi-transparent mirror, Sec. 2.1): the reflected power fraction of a pulse
    at normal incidence is R and the amplitude changes sign (impedance below the medium's),
    from transmission-line theory, r = (Z_L - eta)/(Z_L + eta), independent of the scheme.
    Measured in a dielectric (eps_r 12.96) so that the edge material enters."""
    nx, mid = 1200, 600
    x = np.arange(nx)
    e0 = np.exp(-((x - mid) / 20.0) ** 2) * 1e6
    mats = [W.vacuum(eps_r=12.96)]
    prob = _vacuum_problem(nx, 0.5, 2800, refl=(refl, 0.0), e_init=e0, mats=mats,
                           records=[W.record("e", "e", -1, 1)])
    e = O.Oracle(prob).run()["e"]
    # step 400: the two halves of the split pulse are apart, the left one still inside
    left = np.sum(e[399][:mid] ** 2)
    # step 2800: the left half came back from the left end, the right half left the grid
    back = np.sum(e[2799] ** 2)
    assert abs(back / left - refl) < 0.01 * refl
    peak = e[2799][np.argmax(np.abs(e[2799]))]
    assert peak < 0
    assert abs(abs(peak) / (0.5e6 * math.sqrt(refl)) - 1.0) < 0.02


def test_semi_transparent_end_limits():
    """R -> 1 approaches the perfect conductor, R -> 0 a nearly matched end."""
    nx = 600
    x = np.arange(nx)
    e0 = np.exp(-((x - 300) / 15.0) ** 2) * 1e6
    out = {}
    for refl in (1.0, 1.0 - 1e-8, 1e-8):
        prob = _vacuum_problem(nx, 0.5, 900, refl=(refl, refl), e_init=e0,
                               records=[W.record("e", "e", -1, 1)])
        out[refl] = O.Oracle(prob).run()["e"][-1]
    assert np.max(np.abs(out[1.0 - 1e-8] - out[1.0])) < 1e-3 * 1e6
    assert np.sum(out[1e-8] ** 2) < 1e-3 * np.sum(e0 ** 2)


# ---------------------------------------------------------------- energy exchange with the medium

def _energy_drift(nx, steps, coupling="weak"):
    L = 60e-6
    qm = two_level(2 * math.pi * 2e14, 1e-29 / C["e"], 0.0, 0.0, -1.0, n3d=2e24)
    gam = 0.7
    mats = [W.vacuum(), W.qm_material(qm, overlap=gam)]
    regions = [(0.0, 30e-6, 0), (30e-6, L, 1)]
    dx = L / (nx - 1)
    x = np.arange(nx) * dx
    tau = 20e-15
    e0 = 2e9 * np.exp(-((x - 15e-6) / (C["c0"] * tau)) ** 2) * np.sin(2 * math.pi * 2e14 * x / C["c0"])
    e0[0] = e0[-1] = 0.0
    dt = W.courant_dt(L, nx, C["c0"], 0.5)
    prob = W.make_problem("pt", L, mats, regions, nx, dt, 1, [1.0, 0.0], refl=(1.0, 1.0), e_init=e0,
                          coupling=coupling)
    orc = O.Oracle(prob)
    eps, mu = C["eps0"], C["mu0"]
    h0 = O.describe(qm, C)[0]
    es, hs, us = [], [], []
    for _ in range(steps):
        orc.step()                                  # E^{n+1}, H^{n+1/2}, rho^{n+1/2}
        es.append(orc.e.copy())
        hs.append(orc.h.copy())
        g = orc.groups[0]
        us.append(gam * 2e24 * dx * np.sum(np.real(np.einsum("ij,kji->k", h0, g["rho"]))))
    es, hs, us = np.array(es), np.array(hs), np.array(us)
    # W^{n+1} = eps/2 sum (E^{n+1})^2 dx + mu/2 sum H^{n+3/2} H^{n+1/2} dx ; U^{n+1} ~ mean of halves
    field = 0.5 * eps * dx * np.sum(es[:-1] ** 2, axis=1) + 0.5 * mu * dx * np.sum(hs[1:] * hs[:-1], axis=1)
    # weak coupling: rho^{n+1/2} after step n, averaged to integer times; strong: rho^{n+1}
    atoms = 0.5 * (us[1:] + us[:-1]) if coupling == "weak" else us[:-1]
    total = field + atoms
    return np.max(np.abs(total - total[0])), np.max(np.abs(atoms - atoms[0])), field[0]


def test_poynting_energy_balance_with_two_level_medium():
    """Field energy + Gamma n3D sum tr{H0 rho} dx is conserved without relaxation, up to
    the second-order time discretisation: the polarization current term of eq:efield and
    dP/dt = n3D tr{mu d rho/dt} exchange the energy the systems absorb (this fixes the
    sign and magnitude of the coupling)."""
    d1, ex1, f1 = _energy_drift(600, 3000)
    d2, ex2, _ = _energy_drift(1199, 6000)
    assert ex1 > 0.05 * f1 and abs(ex2 / ex1 - 1) < 0.05
    assert 3.5 < d1 / d2 < 4.5, (d1, d2)
    assert d2 < 2e-3 * ex2


def test_strong_coupling_energy_balance():
    """Strong coupling (Sec. 2.2: rho at the times of E): the same energy exchange between
    field and systems holds to second order."""
    d1, ex1, f1 = _energy_drift(600, 3000, "strong")
    d2, ex2, _ = _energy_drift(1199, 6000, "strong")
    assert ex1 > 0.05 * f1 and abs(ex2 / ex1 - 1) < 0.05
    assert 3.5 < d1 / d2 < 4.5, (d1, d2)
    assert d2 < 2e-3 * ex2


def _coupling_pair(nx, steps):
    """E at 3/4 of a two-level slab driven by a hard Gaussian pulse at the left end, weak and
    strong coupling."""
    L = 40e-6
    qm = two_level(2 * math.pi * 2e14, 2e-29 / C["e"], 1e11, 2e11, -1.0, n3d=3e24)
    mats = [W.vacuum(), W.qm_material(qm)]
    regions = [(0.0, 15e-6, 0), (15e-6, 30e-6, 1), (30e-6, L, 0)]
    dt = W.courant_dt(L, nx, C["c0"], 0.5)
    src = W.source("gauss", 0, 5e9, 2e14, 4.0, 1.0 / 15e-15)
    out = {}
    for cpl in ("weak", "strong"):
        prob = W.make_problem("cpl", L, mats, regions, nx, dt, steps, [1.0, 0.0], refl=(0.0, 0.0),
                              sources=[src], records=[W.record("e", "e", 3 * (nx - 1) // 4, 1)],
                              coupling=cpl)
        out[cpl] = O.run(prob)["e"]
    return out


def test_strong_and_weak_coupling_agree_to_second_order():
    """Both couplings discretise the same equations to second order, so their difference
    falls by 4 when dx and dt are halved (a first-order slip, such as driving rho with E^n
    instead of the midpoint field, would give 2)."""
    a = _coupling_pair(401, 3200)
    b = _coupling_pair(801, 6400)
    d1 = np.max(np.abs(a["strong"] - a["weak"]))
    d2 = np.max(np.abs(b["strong"][1::2] - b["weak"][1::2]))
    scale = np.max(np.abs(a["weak"]))
    assert d1 > 1e-4 * scale            # the schemes really differ
    assert 3.5 < d1 / d2 < 4.6, (d1, d2)


# ---------------------------------------------------------------- Cayley field step

def _cayley(prob):
    prob["field_step"] = "cayley"
    return prob


def test_cayley_field_step_rabi_closed_form():
    """H0 = 0, no relaxation, constant E, mu = mu12 sigma_x: the Cayley transform of
    A = i dt E mu / hbar is diag((1 + i x_j)/(1 - i x_j)) in mu's eigenbasis, x_j = dt E
    lam_j / (2 hbar), i.e. a rotation by 2 atan(x) per step where exp(A) rotates by 2x, so
    rho_22 after n steps is sin^2(2 n atan(mu12 E dt / (2 hbar)))."""
    z21 = 1e-10
    qm = two_level(0.0, z21, 0.0, 0.0, -1.0)
    mu12 = C["e"] * z21
    dt, nt = 5e-16, 400
    e_c = 0.6 * HB / (mu12 * dt)                      # x = 0.3 per level
    recs = O.Oracle(_cayley(single_point(qm, nt, dt, [1.0, 0.0], e_const=e_c))).run()
    n = np.arange(nt) + 1
    x = mu12 * e_c * dt / (2 * HB)
    cay = np.sin(2 * n * math.atan(x)) ** 2
    exact = np.sin(2 * n * x) ** 2
    assert np.max(np.abs(recs["p1"] - cay)) < 1e-12
    assert np.max(np.abs(recs["p1"] - exact)) > 0.1    # the two field steps really differ


@pytest.mark.parametrize("n", [3, 4])
def test_cayley_field_step_keeps_density_matrices_valid(n):
    """The Cayley transform of an anti-Hermitian matrix is unitary: trace one, Hermitian,
    positive semi-definite density matrices in every quantum cell (Sec. 2.2)."""
    prob = _cayley(W.random_small(40 + n, N=n, nx=30, n_steps=60, full_records=False))
    prob["e_init"] = np.full(30, 3e9)                # strong field: large Cayley angles
    orc = O.Oracle(prob)
    for _ in range(60):
        orc.step()
        for g in orc.groups:
            rho = g["rho"]
            assert np.max(np.abs(np.trace(rho, axis1=1, axis2=2) - 1.0)) < 1e-12
            assert np.max(np.abs(rho - np.conj(np.transpose(rho, (0, 2, 1))))) < 1e-14
            assert np.linalg.eigvalsh(rho).min() > -1e-12


def test_cayley_and_exact_field_steps_agree_to_second_order():
    """Detuned Rabi problem: the Cayley and exact field steps differ by O(dt^2), so the
    difference of their trajectories at fixed times falls by 4 when dt halves."""
    om, z21 = 2 * math.pi * 1e14, 1e-29 / C["e"]
    e_c = 0.25 * HB * om / 1e-29
    qm = two_level(om, z21, 0.0, 0.0, -1.0)

    def diff(dt):
        nt = int(round(1e-13 / dt))
        a = O.Oracle(single_point(qm, nt, dt, [1.0, 0.0], e_const=e_c)).run()["p1"]
        b = O.Oracle(_cayley(single_point(qm, nt, dt, [1.0, 0.0], e_const=e_c))).run()["p1"]
        return a - b

    d1 = diff(2e-16)
    d2 = diff(1e-16)[1::2]
    r = np.max(np.abs(d1)) / np.max(np.abs(d2))
    assert np.max(np.abs(d1)) > 1e-6
    assert 3.6 < r < 4.4, r


# ---------------------------------------------------------------- P9 self-induced transparency

@pytest.mark.slow
def test_p9_self_induced_transparency():
    """A 2 pi sech pulse crosses the two-level medium with its energy and leaves the
    systems in the ground state; a pi pulse is absorbed (area theorem, Sec. 4.1)."""
    r2 = O.run(W.sit_2lvl(area_pi=2.0))
    r1 = O.run(W.sit_2lvl(area_pi=1.0))
    en2 = [np.sum(r2[f"e@{c}"] ** 2) for c in (300, 750, 1199)]
    en1 = [np.sum(r1[f"e@{c}"] ** 2) for c in (300, 750, 1199)]
    assert en2[2] / en2[0] > 0.97
    for c in (300, 750, 1199):
        assert r2[f"inv@{c}"].max() > 0.99          # fully inverted once
        assert r2[f"inv@{c}"][-1] < -0.99           # returned to the ground state
    assert en1[2] / en1[0] < 0.75


# ---------------------------------------------------------------- P10 algebra of the description

def test_p10a_two_level_round_trip():
    """qm_desc_2lvl: R = gamma1/2 [[0, 1-w0], [1+w0, 0]], gamma_12,p = gamma2 - gamma1/2;
    gamma1 = gamma12 + gamma21, w0 = (gamma21 - gamma12)/(gamma21 + gamma12),
    gamma2 = (gamma12 + gamma21)/2 + gamma_12,p (Sec. 3.1.1)."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        g1, g2, w0 = rng.uniform(1e9, 1e13), rng.uniform(1e9, 1e13), rng.uniform(-1, 1)
        h0, mu, rates, deph = O.two_level_description(two_level(1e14, 1e-10, g1, g2, w0), C)
        g12, g21 = rates[0, 1], rates[1, 0]
        assert abs((g12 + g21) / g1 - 1) < 1e-14
        assert abs((g21 - g12) / (g21 + g12) - w0) < 1e-13
        assert abs(((g12 + g21) / 2 + deph[0]) / g2 - 1) < 1e-14
        assert abs((h0[1, 1] - h0[0, 0]).real / HB - 1e14) < 1e-2
        assert abs(mu[0, 1] + C["e"] * 1e-10) < 1e-40


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_p10b_rate_form_equals_lindblad_form(n):
    rng = np.random.default_rng(100 + n)
    qm = W.random_qm(rng, n)
    _, _, rates, deph, _ = O.describe(qm, C)
    ops, lam_min = O.lindblad_from_rates(rates, deph)
    assert lam_min > -1e-6 * deph.max()
    for _ in range(3):
        rd, ro = W.random_rho(rng, n)
        rho = O.unpack_hermitian(rd, ro)
        a = O.dissipator(rho, rates, deph)
        b = O.lindblad_dissipator(rho, ops)
        assert np.max(np.abs(a - b)) < 1e-9 * np.max(np.abs(a))


def test_p10c_non_euclidean_dephasing_is_flagged():
    """Pure dephasing rates need a positive semi-definite C (Sec. 3.1.1, eq:puredeph)."""
    assert O.is_completely_positive(np.array([1e12, 1e12, 1e12]), 3)
    assert O.is_completely_positive(np.array([1e12, 4e12, 1e12]), 3)   # collinear: 1, 2, 1
    assert not O.is_completely_positive(np.array([1e12, 1e12, 10e12]), 3)


# ---------------------------------------------------------------- P11 the paper's printed numbers
# (read from tests/golden/, see the golden-fixture tests at the end of this file)

# ---------------------------------------------------------------- explicit Lindblad operators

def test_explicit_lindblad_ops_closed_form():
    """Decay L1 = sqrt(g)|0><1| and dephasing L2 = sqrt(k)|1><1| (eq:lindbladdiss) on a
    single point without field: rho_11 = rho_11(0) e^{-g t} and
    rho_01 = rho_01(0) e^{(i w - (g + k)/2) t} for H0 = diag(0, hbar w)."""
    hbar = C["hbar"]
    w, g, k = 2 * np.pi * 1e13, 1.0e12, 2.5e12
    qm = W.general_qm(1e24, [0.0, hbar * w], None, None, np.array([1e-29]), np.zeros((2, 2)), [0.0])
    l1 = np.zeros((2, 2), complex)
    l1[0, 1] = np.sqrt(g)
    l2 = np.zeros((2, 2), complex)
    l2[1, 1] = np.sqrt(k)
    qm["lindblad_ops"] = [l1, l2]
    rho01 = 0.3 + 0.1j
    dt, steps = 1e-15, 500
    prob = W.make_problem("lops", 0.0, [W.qm_material(qm)], [(0.0, 0.0, 0)], 1, dt, steps,
                          [0.4, 0.6], [rho01])
    orc = O.Oracle(prob)
    for n in range(1, steps + 1):
        orc.step()
        if n % 100:
            continue
        rho = orc.density_at(0)
        t = n * dt
        assert abs(rho[1, 1].real - 0.6 * np.exp(-g * t)) < 1e-12
        assert abs(rho[0, 0].real - (1.0 - 0.6 * np.exp(-g * t))) < 1e-12
        assert abs(rho[0, 1] - rho01 * np.exp((1j * w - 0.5 * (g + k)) * t)) < 1e-12
    # and the rate form with the same physics: gamma_01 = g, no rate 0 -> 1, and the
    # coherence decay (g + k)/2 = g/2 + gamma_p gives gamma_p = k/2
    qr = W.general_qm(1e24, [0.0, hbar * w], None, None, np.array([1e-29]),
                      np.array([[0.0, g], [0.0, 0.0]]), [k / 2])
    pr = W.make_problem("rates", 0.0, [W.qm_material(qr)], [(0.0, 0.0, 0)], 1, dt, steps,
                        [0.4, 0.6], [rho01])
    o2 = O.Oracle(pr)
    for _ in range(steps):
        o2.step()
    assert np.max(np.abs(o2.density_at(0) - orc.density_at(0))) < 1e-12


@pytest.mark.parametrize("n,seed", [(3, 61), (4, 62)])
def test_explicit_lindblad_ops_equal_rate_form(n, seed):
    """The rate-form dissipator (eq:relax_pop and the dephasing law) and the operator form
    (eq:lindbladdiss) with the equivalent jump and dephasing operators give the same run
    of a driven device (fields, populations, coherences)."""
    prob = W.random_small(seed, N=n, nx=30, n_steps=80, n_materials=1)
    qm = prob["materials"][1]["qm"]
    ops, lam_min = O.lindblad_from_rates(np.asarray(qm["rates"]), np.asarray(qm["pure_deph"]))
    assert lam_min >= -1e-9 * np.abs(qm["pure_deph"]).max()     # completely positive case
    ref = O.run(prob)
    qm2 = dict(qm)
    qm2["lindblad_ops"] = ops
    prob2 = dict(prob)
    prob2["materials"] = [prob["materials"][0], dict(prob["materials"][1], qm=qm2)]
    got = O.run(prob2)
    for key in ref:
        scale = max(1e-30, np.abs(ref[key]).max())
        assert np.max(np.abs(np.asarray(got[key]) - np.asarray(ref[key]))) <= 1e-10 * scale, key


# ---------------------------------------------------------------- golden fixtures (printed examples)

GOLDEN = __import__("pathlib").Path(__file__).parent / "golden"


def _golden(name):
    """key -> list of floats from a fixture of the paper's printed example values."""
    out = {}
    for line in (GOLDEN / name).read_text().splitlines():
        line = line.split("#", 1)[0].strip()
        if line:
            key, val = line.split("=", 1)
            out[key.strip()] = [float(v) for v in val.split()]
    return out


def test_golden_sit_listing():
    """Sec. 4.1 listing: the transition frequency is 2 pi 2e14, the sech source carries a
    2 pi pulse area for the dipole e z21, and the two-level constructor relaxes the
    inversion towards w0 at the rate gamma1 (closed form, single point, no field)."""
    g = _golden("sit_ziolkowski.txt")
    assert g["omega21"][0] == 2 * math.pi * 2e14
    amp, freq, shift, width = g["source"]
    src = W.source("sech", 0, amp, 0.0, shift, width, phase=math.pi / 2)
    t = np.linspace(-50e-15, 250e-15, 300001)
    env = np.array([O.source_value(src, tt) for tt in t])
    area = C["e"] * g["z21"][0] / HB * np.trapezoid(env, t)
    assert abs(area / (2 * math.pi) - 1.0) < 1e-3
    assert abs(t[np.argmax(env)] - shift / width) < 1e-17     # envelope peak at 50 fs
    qm = W.two_level_params(g["n3d"][0], g["omega21"][0], g["z21"][0], g["gamma1"][0], g["gamma2"][0], g["w0"][0])
    dt, steps = 2e-12, 50
    prob = W.make_problem("sit-relax", 0.0, [W.qm_material(qm)], [(0.0, 0.0, 0)], 1, dt, steps, [0.0, 1.0])
    orc = O.Oracle(prob)
    for _ in range(steps):
        orc.step()
    rho = orc.density_at(0)
    w = (rho[1, 1] - rho[0, 0]).real
    w0, g1 = g["w0"][0], g["gamma1"][0]
    assert abs(w - (w0 + (1.0 - w0) * math.exp(-g1 * steps * dt))) < 1e-12


def test_golden_qcl_listing_is_the_workload():
    """Sec. 4.4 listing: the five-level comb workload holds the printed Hamiltonian,
    dipole, rate matrix, dephasing, density, material, mirrors and length; with column
    packing the dipole couples (3,4) and the tunnelling (1,3), (2,3)."""
    g = _golden("qcl_tzenov.txt")
    e = C["e"]
    prob = W.qcl5_comb(nx=64, n_steps=10)
    qm = prob["materials"][0]["qm"]
    assert np.array_equal(qm["h0_diag"], np.array(g["h0_diag_ev"]) * e)
    assert np.array_equal(qm["h0_off"], np.array(g["h0_off_ev"]) * e)
    assert np.array_equal(qm["mu_off"], np.array(g["mu_off_em"]) * e)
    rates = np.array([g[f"rates_row{k}"] for k in range(1, 6)])
    assert np.array_equal(qm["rates"], rates)
    tau = np.array(g["dephasing_times"])
    assert np.allclose(qm["pure_deph"], np.where(tau > 0, 1.0 / np.where(tau > 0, tau, 1.0), 0.0), rtol=1e-15)
    assert qm["n3d"] == g["n3d"][0]
    m = prob["materials"][0]
    assert [m["eps_r"], m["overlap"], m["alpha0"]] == g["material"]
    assert list(prob["refl"]) == g["reflectivity"] and prob["length"] == g["length"][0]
    h = O.unpack_hermitian(qm["h0_diag"], qm["h0_off"])
    u = O.unpack_hermitian([0.0] * 5, qm["mu_off"])
    assert [(i, j) for i in range(5) for j in range(i + 1, 5) if u[i, j] != 0] == [(2, 3)]
    assert [(i, j) for i in range(5) for j in range(i + 1, 5) if h[i, j] != 0] == [(0, 2), (1, 2)]


def test_golden_ladder_levels():
    """Sec. 4.3: the ladder workload's level spacings are the printed formula's, and w0 is
    the E_3 -> E_4 transition frequency as the text states."""
    g = _golden("ladder_marskar.txt")
    n = int(g["levels"][0])
    qm = W.ladder(n, nx=64, n_steps=10)["materials"][1]["qm"]
    gaps = np.diff(np.asarray(qm["h0_diag"])) / (HB * g["omega0"][0])
    assert np.allclose(gaps, g["spacings"], rtol=1e-12)
    assert abs(gaps[2] - 1.0) < 1e-12


# ---------------------------------------------------------------- sources and regions

def _envelope(kind, amp, shift, width, period=0.0, count=1):
    """The oracle's source with its carrier set to 1 (frequency 0, phase pi/2): the envelope."""
    return W.source(kind, 0.0, amp, 0.0, shift, width, phase=math.pi / 2, period=period, count=count)


def test_gaussian_source_closed_forms():
    """Gaussian source of Sec. 2.1/3.1 (the paper gives no formula; reading: amplitude
    times exp(-(width t - shift)^2) times the carrier): the envelope integrates to
    amp sqrt(pi)/width, peaks at t = shift/width with the value amp, falls to amp/e one
    1/width either side of the peak, and the carrier is sin(2 pi f t + phase) of the
    absolute time."""
    amp, shift, width = 3.7e8, 5.0, 1.0 / 30e-15
    src = _envelope("gauss", amp, shift, width)
    t = np.linspace(0.0, 2 * shift / width, 400001)
    env = np.array([O.source_value(src, tt) for tt in t])
    area = np.trapezoid(env, t)
    assert abs(area / (amp * math.sqrt(math.pi) / width) - 1.0) < 1e-9
    tp = shift / width
    assert abs(O.source_value(src, tp) - amp) < 1e-15 * amp
    assert abs(t[np.argmax(env)] - tp) < 1e-18
    for d in (-1.0, 1.0):
        assert abs(O.source_value(src, tp + d / width) - amp / math.e) < 1e-14 * amp
    # carrier: at the peak the value is amp sin(2 pi f tp + phase), whatever f and phase
    f, ph = 1.9e14, 0.7
    s2 = W.source("gauss", 0.0, amp, f, shift, width, phase=ph)
    assert abs(O.source_value(s2, tp) - amp * math.sin(2 * math.pi * f * tp + ph)) < 1e-14 * amp


def test_pulse_train_is_a_sum_of_shifted_pulses():
    """A train of `count` pulses with period T: its envelope is the sum of the single
    pulse's envelope shifted by 0, T, 2T, ... (peaks at shift/width + q T); the carrier
    stays that of the absolute time."""
    amp, shift, width, T = 2.0e8, 4.0, 1.0 / 20e-15, 1.5e-12
    single = _envelope("gauss", amp, shift, width)
    train = _envelope("gauss", amp, shift, width, period=T, count=3)
    for t in np.linspace(-0.2e-12, 5e-12, 2001):
        want = sum(O.source_value(single, t - q * T) for q in range(3))
        assert abs(O.source_value(train, t) - want) <= 1e-15 * amp
    for q in range(3):
        assert abs(O.source_value(train, shift / width + q * T) - amp) < 1e-12 * amp
    # beyond the last pulse the train is the single pulse's tail only
    assert O.source_value(train, shift / width + 3 * T) < 1e-100
    st = _envelope("sech", amp, shift, width, period=T, count=2)
    ss = _envelope("sech", amp, shift, width)
    for t in np.linspace(0.0, 3e-12, 301):
        assert abs(O.source_value(st, t) - O.source_value(ss, t) - O.source_value(ss, t - T)) <= 1e-15 * amp


def test_lambda_drive_is_a_pi_half_pulse_train():
    """The three-level Lambda workload's drive: each Gaussian of the train carries the
    pulse area pi/2 on a 1e-29 C m dipole (area = dipole/hbar times the envelope
    integral), its first peak is at 100 fs and the period is 2 ps."""
    prob = W.lambda3(nx=64, n_steps=10)
    s = prob["sources"][0]
    env = _envelope("gauss", s["amp"], s["shift"], s["width"])
    t = np.linspace(-200e-15, 400e-15, 600001)      # +- 10 widths around the first peak
    area = 1e-29 / HB * np.trapezoid([O.source_value(env, tt) for tt in t], t)
    assert abs(area / (math.pi / 2) - 1.0) < 1e-6
    assert abs(s["shift"] / s["width"] - 100e-15) < 1e-27
    assert s["period"] == 2e-12 and s["kind"] == "gauss" and s["freq"] == 190e12


def test_region_lookup_at_interfaces():
    """Regions are half-open [x_start, x_end) (reading of Sec. 3.1, region): a node on an
    interface belongs to the region that starts there, the node at the far end to the
    last region, a node beyond the end by less than dx/2 to the right-most region, and a
    node in no region is an error."""
    dx = 0.25
    regions = [dict(x_start=0.0, x_end=1.0, material=0), dict(x_start=1.0, x_end=2.0, material=1),
               dict(x_start=2.0, x_end=3.0, material=2)]
    got = [O.material_index(regions, m * dx, dx) for m in range(13)]
    assert got == [0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 2, 2, 2]
    assert O.material_index(regions, 3.0 + 0.4 * dx, dx) == 2
    with pytest.raises(ValueError):
        O.material_index(regions, 3.0 + 0.6 * dx, dx)
    gap = [dict(x_start=0.0, x_end=1.0, material=0), dict(x_start=1.5, x_end=3.0, material=1)]
    with pytest.raises(ValueError):
        O.material_index(gap, 1.25, dx)
    # a solve sees the same split: E nodes on the interfaces carry the right-hand medium
    p = W.lambda3(nx=65, n_steps=1, n_regions=4)
    orc = O.Oracle(p)
    assert list(orc.mat_e[[0, 15, 16, 17, 31, 32, 48, 64]]) == [0, 0, 1, 1, 1, 2, 3, 3]


def test_source_position_rounds_to_the_nearest_node():
    """Source positions are converted to grid nodes by round(x/dx), ties to the even node
    (Sec. 3.2: positions are converted to integer grid indices)."""
    nx, length = 11, 1e-6
    dx = length / (nx - 1)
    for x, cell in ((0.0, 0), (0.49 * dx, 0), (0.5 * dx, 0), (1.5 * dx, 2), (2.5 * dx, 2), (3.51 * dx, 4),
                    (length, 10)):
        assert O.source_cell(x, dx, nx) == cell, (x / dx, cell)
    for bad in (-0.6 * dx, length + 0.6 * dx):
        with pytest.raises(ValueError):
            O.source_cell(bad, dx, nx)
