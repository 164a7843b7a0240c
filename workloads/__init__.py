"""Seeded synthetic inputs for the 1D Maxwell-Bloch hot path.

This module only builds *inputs*: device and scenario descriptions made of
plain numbers and numpy arrays.  It holds none of the method's arithmetic
(no Liouvillian, no propagator, no FDTD coefficient, no source waveform) so
that the oracle under ``oracle/`` and the HIP library can both consume the
same description without sharing any numerics.

A *problem* is a dict:

``consts``     SI constants (CODATA 2018): hbar, e, c0, mu0, eps0.
``length``     device length L [m] (the grid spacing is L/(nx-1)).
``refl``       (R_left, R_right) field reflectivity of the two ends, each in [0, 1].
``coupling``   "weak" (density matrix half a step after E, the default) or "strong"
               (density matrix at the same times as E).
``materials``  list of dicts: eps_r, mu_r, alpha0 [1/m], overlap (Gamma) and
               ``qm`` = None (no quantum system) or a dict with n3d [m^-3],
               h0_diag (N,) [J], h0_off (N(N-1)/2,) complex [J], mu_diag,
               mu_off [C m], rates (N,N) with rates[i, j] = gamma_ij = rate of
               scattering from level j to level i (diagonal ignored), and
               pure_deph (N(N-1)/2,) [1/s].  Off-diagonal vectors use the
               packing of the upper triangle by columns:
               (1,2), (1,3), (2,3), (1,4), (2,4), (3,4), ...
``regions``    list of dicts x_start, x_end [m], material (index).
``nx``, ``dt`` [s], ``n_steps``, ``precision`` (64 or 32).
``rho_diag``, ``rho_off``  initial density matrix in the same packed form.
``e_init``     None (zero field) or an (nx,) array of initial E [V/m].
``sources``    list of dicts: kind ('sech'|'gauss'|'table'), hard (bool), x
               (position [m]; each consumer converts it to the nearest E node),
               amp [V/m], freq [Hz], shift, width [1/s], phase [rad],
               period [s], count (number of pulses in a train).
``records``    list of dicts: name, quantity ('e'|'h'|'pop'|'inv'|'rho_re'|
               'rho_im'), i, j (0-based levels), cell (-1 = whole domain),
               interval (steps).

Seeds are fixed per configuration: base 20050541 plus the configuration
index.  Random draws that the method itself needs (the noise initial field)
are made here and passed in as ``e_init``.
"""
from __future__ import annotations

import math
import numpy as np

SEED_BASE = 20050541

CODATA = {
    "hbar": 1.054571817e-34,
    "e": 1.602176634e-19,
    "c0": 299792458.0,
    "mu0": 1.25663706212e-6,
}
CODATA["eps0"] = 1.0 / (CODATA["mu0"] * CODATA["c0"] ** 2)

QUANTITIES = ("e", "h", "pop", "inv", "rho_re", "rho_im")


def n_off(n: int) -> int:
    return n * (n - 1) // 2


def vacuum(eps_r=1.0, mu_r=1.0, alpha0=0.0, overlap=1.0):
    return {"eps_r": float(eps_r), "mu_r": float(mu_r), "alpha0": float(alpha0),
            "overlap": float(overlap), "qm": None}


def qm_material(qm, eps_r=1.0, mu_r=1.0, alpha0=0.0, overlap=1.0):
    m = vacuum(eps_r, mu_r, alpha0, overlap)
    m["qm"] = qm
    return m


def two_level_params(n3d, omega21, z21, gamma1, gamma2, w0, consts=CODATA):
    """Parameters of the simplified two-level constructor, returned raw.

    The conversion into H0, mu, R and the pure dephasing rate is done by each
    consumer (the oracle and the library) on its own; the generator only
    records the six numbers.
    """
    return {"kind": "2lvl", "n3d": float(n3d), "omega21": float(omega21),
            "z21": float(z21), "gamma1": float(gamma1), "gamma2": float(gamma2),
            "w0": float(w0)}


def general_qm(n3d, h0_diag, h0_off, mu_diag, mu_off, rates, pure_deph):
    n = len(h0_diag)
    h0_off = np.zeros(n_off(n), complex) if h0_off is None else np.asarray(h0_off, complex)
    mu_off = np.zeros(n_off(n), complex) if mu_off is None else np.asarray(mu_off, complex)
    mu_diag = np.zeros(n) if mu_diag is None else np.asarray(mu_diag, float)
    qm = {"kind": "general", "n3d": float(n3d),
          "h0_diag": np.asarray(h0_diag, float), "h0_off": h0_off,
          "mu_diag": mu_diag, "mu_off": mu_off,
          "rates": np.asarray(rates, float).reshape(n, n),
          "pure_deph": np.asarray(pure_deph, float).reshape(n_off(n))}
    assert qm["h0_off"].shape == (n_off(n),) and qm["mu_off"].shape == (n_off(n),)
    return qm


def qm_levels(qm) -> int:
    if qm is None:
        return 0
    if qm["kind"] == "2lvl":
        return 2
    return len(qm["h0_diag"])


def problem_levels(p) -> int:
    ns = {qm_levels(m["qm"]) for m in p["materials"] if m["qm"] is not None}
    assert len(ns) <= 1, "all quantum materials of one device share one level count"
    return ns.pop() if ns else 0


def node_x(length, nx, cell):
    """Position [m] of E node `cell` of an nx-node grid over `length` (x_m = m dx)."""
    return 0.0 if nx <= 1 else cell * (length / (nx - 1))


def source(kind, x, amp, freq, shift, width, phase=0.0, hard=True, period=0.0, count=1):
    """A source at position x [m] (hard: sets E there, soft: adds to it)."""
    return {"kind": kind, "hard": bool(hard), "x": float(x), "amp": float(amp),
            "freq": float(freq), "shift": float(shift), "width": float(width),
            "phase": float(phase), "period": float(period), "count": int(count)}


def table_source(x, values, hard=True):
    """Sampled waveform at position x [m]: values[n] at t_n = n dt, zero after the table."""
    s = source("table", x, 0.0, 0.0, 0.0, 0.0, hard=hard)
    s["table"] = np.asarray(values, float)
    return s


def record(name, quantity, cell, interval, i=0, j=0):
    assert quantity in QUANTITIES
    return {"name": name, "quantity": quantity, "cell": int(cell),
            "interval": int(interval), "i": int(i), "j": int(j)}


def make_problem(name, length, materials, regions, nx, dt, n_steps, rho_diag,
                 rho_off=None, refl=(0.0, 0.0), e_init=None, sources=(), records=(),
                 precision=64, consts=CODATA, coupling="weak", field_step="exact"):
    n = len(rho_diag)
    assert coupling in ("weak", "strong")
    assert field_step in ("exact", "cayley")
    return {"name": name, "consts": dict(consts), "length": float(length), "coupling": coupling,
            "field_step": field_step,
            "refl": (float(refl[0]), float(refl[1])), "materials": list(materials),
            "regions": [dict(x_start=float(a), x_end=float(b), material=int(m)) for a, b, m in regions],
            "nx": int(nx), "dt": float(dt), "n_steps": int(n_steps), "precision": int(precision),
            "rho_diag": np.asarray(rho_diag, float),
            "rho_off": np.zeros(n_off(n), complex) if rho_off is None else np.asarray(rho_off, complex),
            "e_init": None if e_init is None else np.asarray(e_init, float),
            "sources": list(sources), "records": list(records)}


def courant_dt(length, nx, c_max, courant=0.5):
    """Time step dt = C * dx / c_max with dx = L/(nx-1)."""
    return courant * (length / (nx - 1)) / c_max


def splitmix64_uniform(seed: int, n: int) -> np.ndarray:
    """n uniform doubles in [0,1) from the SplitMix64 counter-based stream."""
    mask = (1 << 64) - 1
    out = np.empty(n)
    state = seed & mask
    for k in range(n):
        state = (state + 0x9E3779B97F4A7C15) & mask
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        z = z ^ (z >> 31)
        out[k] = (z >> 11) * (1.0 / 9007199254740992.0)
    return out


# ---------------------------------------------------------------------------
# Benchmark configurations
# ---------------------------------------------------------------------------

def sit_2lvl(nx=1500, n_steps=20000, precision=64, area_pi=2.0, probes=(300, 750, 1199),
             rec_interval=1):
    """Two-level self-induced transparency: 150 um, medium in the central 100 um.

    omega0 = 2 pi 2e14 rad/s, dipole 1e-29 C m, n3d = 1e24 m^-3, T1 = T2 = 1 ns
    (gamma1 = gamma2 = 1e9 1/s), ground state start (w0 = -1), hard sech at the
    left end with 100 fs intensity FWHM, carrier 200 THz, area ``area_pi`` * pi.
    Right end absorbing (R = 0), Courant number 1/2.
    """
    c = CODATA
    L = 150e-6
    dipole = 1e-29
    qm = two_level_params(1e24, 2 * math.pi * 2e14, dipole / c["e"], 1e9, 1e9, -1.0)
    mats = [vacuum(), qm_material(qm)]
    regions = [(0.0, 25e-6, 0), (25e-6, 125e-6, 1), (125e-6, L, 0)]
    dt = courant_dt(L, nx, c["c0"])
    fwhm = 100e-15
    tau = fwhm / (2.0 * math.acosh(math.sqrt(2.0)))   # intensity FWHM of sech^2
    amp = area_pi * c["hbar"] / (dipole * tau)         # area = mu A pi tau / hbar
    src = source("sech", 0.0, amp, 2e14, 10.0, 1.0 / tau)
    recs = []
    for p in probes:
        recs.append(record(f"e@{p}", "e", p, rec_interval))
        recs.append(record(f"inv@{p}", "inv", p, rec_interval, i=0, j=1))
    return make_problem("sit-2lvl", L, mats, regions, nx, dt, n_steps, [1.0, 0.0],
                        refl=(0.0, 0.0), sources=[src], records=recs, precision=precision)


def _lambda3_material(rng, c):
    """One seeded three-level Lambda medium (levels 1, 2 low; 3 high)."""
    h = 2 * math.pi * c["hbar"]
    d13, d23 = rng.uniform(-2e12, 2e12, 2)
    e3 = h * (200e12 + d13)
    e2 = e3 - h * (180e12 + d23)
    mu13, mu23 = 1e-29 * rng.uniform(0.5, 1.5, 2)
    g31, g32 = rng.uniform(0.1e12, 1e12, 2)           # 3 -> 1, 3 -> 2
    g12 = rng.uniform(0.01e12, 0.1e12)                # 2 <-> 1
    rates = np.zeros((3, 3))
    rates[0, 2] = g31          # gamma_13: from 3 into 1
    rates[1, 2] = g32          # gamma_23: from 3 into 2
    rates[0, 1] = g12          # gamma_12: from 2 into 1
    rates[1, 0] = g12          # gamma_21: from 1 into 2
    # pure dephasing built as a sum of two squared-distance patterns so that it
    # is always a valid (Euclidean) dephasing set: common part + (u_i-u_j)^2/2
    base = rng.uniform(1e12, 5e12)
    u = rng.uniform(0.0, math.sqrt(8e12), 3)
    deph = np.array([base + 0.5 * (u[0] - u[1]) ** 2,      # (1,2)
                     base + 0.5 * (u[0] - u[2]) ** 2,      # (1,3)
                     base + 0.5 * (u[1] - u[2]) ** 2])     # (2,3)
    mu_off = np.array([0.0, mu13, mu23], complex)         # (1,2), (1,3), (2,3)
    return general_qm(1e24, [0.0, e2, e3], None, None, mu_off, rates, deph)


def lambda3(nx=32768, n_steps=200000, precision=64, n_regions=16, n_probes=64,
            rec_interval=10, seed=None):
    """Three-level Lambda medium over a 2 mm grid, 16 seeded materials.

    Transitions at 2 pi {180, 200} THz with random detunings, Gaussian pulse
    train drive (tau 30 fs, period 2 ps, first peak at 100 fs, carrier 190 THz,
    pi/2 area on a 1e-29 C m dipole), populations recorded at 64 probes every
    10 steps.  Both ends absorbing.
    """
    c = CODATA
    rng = np.random.default_rng(SEED_BASE + 1 if seed is None else seed)
    L = 2e-3
    mats = [_lambda3_material(rng, c) for _ in range(n_regions)]
    mats = [qm_material(q) for q in mats]
    edges = np.linspace(0.0, L, n_regions + 1)
    regions = [(edges[k], edges[k + 1], k) for k in range(n_regions)]
    dt = courant_dt(L, nx, c["c0"])
    tau = 30e-15
    amp = math.sqrt(math.pi) * c["hbar"] / (2 * 1e-29 * tau)
    src = source("gauss", 0.0, amp, 190e12, 100e-15 / tau, 1.0 / tau, period=2e-12,
                 count=max(1, int(math.ceil(n_steps * dt / 2e-12)) + 1))
    recs = []
    for k in range(n_probes):
        cell = int(round((k + 0.5) * nx / n_probes))
        for lvl in range(3):
            recs.append(record(f"rho{lvl}{lvl}@{cell}", "pop", cell, rec_interval, i=lvl, j=lvl))
    return make_problem("lambda-3lvl", L, mats, regions, nx, dt, n_steps, [0.5, 0.5, 0.0],
                        refl=(0.0, 0.0), sources=[src], records=recs, precision=precision)


def qcl6(nx=8192, n_steps=1_000_000, precision=32, seed=None, rec_interval=1):
    """QCL-like six-level active region in a 2 mm cavity with reflecting ends.

    Background eps_r = 12.96, overlap 0.9, alpha0 = 1100 1/m; sorted energies
    U(0, 200) meV with E1 = 0 plus two tunnelling couplings; real symmetric
    dipoles e * U(-4, 4) nm; 15 downward scattering rates U(0.1, 2) 1/ps; pure
    dephasing 1/ps on every pair; n3d = 5.6e21 m^-3; start in the top level;
    noise initial field of amplitude 1 V/m; E recorded next to the right facet.
    """
    c = CODATA
    rng = np.random.default_rng(SEED_BASE + 2 if seed is None else seed)
    N = 6
    meV = 1e-3 * c["e"]
    en = np.sort(np.concatenate([[0.0], rng.uniform(0.0, 200.0, N - 1)])) * meV
    gaps = np.diff(en)
    h0_off = np.zeros(n_off(N), complex)
    order = np.argsort(gaps)[:2]
    for k in order:                        # couple the two closest adjacent pairs
        i, j = k, k + 1                    # 0-based, i < j
        idx = j * (j - 1) // 2 + i
        h0_off[idx] = rng.uniform(0.5, 1.5) * meV
    mu_off = np.array(c["e"] * rng.uniform(-4e-9, 4e-9, n_off(N)), complex)
    rates = np.zeros((N, N))
    for j in range(N):
        for i in range(j):
            rates[i, j] = rng.uniform(0.1e12, 2e12)     # from upper j into lower i
    deph = np.full(n_off(N), 1e12)
    qm = general_qm(5.6e21, en, h0_off, None, mu_off, rates, deph)
    L = 2e-3
    mats = [qm_material(qm, eps_r=12.96, overlap=0.9, alpha0=1100.0)]
    dt = courant_dt(L, nx, c["c0"] / math.sqrt(12.96))
    u = splitmix64_uniform(SEED_BASE + 2, nx)
    e_init = 1.0 * (2.0 * u - 1.0)
    e_init[0] = 0.0
    e_init[-1] = 0.0
    recs = [record("e@facet", "e", nx - 2, rec_interval)]
    rho = np.zeros(N)
    rho[N - 1] = 1.0
    return make_problem("qcl-6lvl", L, mats, [(0.0, L, 0)], nx, dt, n_steps, rho,
                        refl=(1.0, 1.0), e_init=e_init, records=recs, precision=precision)


def qcl5_comb(nx=8192, n_steps=200_000, precision=32, rec_interval=1, noise=1.0):
    """The paper's quantum cascade laser frequency-comb example (Sec. 4.4, its C++ listing).

    Five-level active region with the printed Hamiltonian (diagonal energies and the two
    tunnelling couplings (1,3), (2,3), in eV), the single dipole element on the (3,4)
    upper/lower laser transition (-e * 4 nm), the printed 5 x 5 scattering-rate matrix
    (entry [i][j] read as the rate from level j into level i, the index order of the
    population equation of Sec. 3.1.1), pure dephasing 1/(0.6 ps) on the injector pairs
    (1,3), (2,3) and 1/(1 ps) elsewhere, n3d = 5.6e21 m^-3, background eps_r 12.96,
    overlap 0.9, alpha0 1100 1/m, a 5 mm cavity with semi-transparent mirrors R = 0.8 at
    both ends, all population in level 3, and the field at the left facet recorded.
    The listing leaves the grid, the end time and the noise of the random initial field
    open: nx cells at Courant 1/2, n_steps steps, uniform noise of amplitude `noise` V/m
    from SplitMix64.
    """
    c = CODATA
    ev = c["e"]
    N = 5
    en = np.array([0.10103, 0.09677, 0.09720, 0.08129, 0.07633]) * ev
    h0_off = np.zeros(n_off(N), complex)
    h0_off[1] = 1.2329e-3 * ev                   # (1,3)
    h0_off[2] = -1.3447e-3 * ev                  # (2,3)
    mu_off = np.zeros(n_off(N), complex)
    mu_off[5] = -ev * 4e-9                       # (3,4)
    rates = np.array([[0.0000000, 0.4947e12, 0.0974e12, 0.8116e12, 1.0410e12],
                      [0.8245e12, 0.0000000, 0.1358e12, 0.6621e12, 1.1240e12],
                      [0.0229e12, 0.0469e12, 0.0000000, 0.0794e12, 0.0357e12],
                      [0.0047e12, 0.0029e12, 0.1252e12, 0.0000000, 0.2810e12],
                      [0.0049e12, 0.0049e12, 0.1101e12, 0.4949e12, 0.0000000]])
    inj, other = 1.0 / 0.6e-12, 1.0 / 1.0e-12
    deph = np.array([0.0, inj, inj] + [other] * 7)
    qm = general_qm(5.6e21, en, h0_off, None, mu_off, rates, deph)
    L = 5e-3
    mats = [qm_material(qm, eps_r=12.96, overlap=0.9, alpha0=1100.0)]
    dt = courant_dt(L, nx, c["c0"] / math.sqrt(12.96))
    e_init = noise * (2.0 * splitmix64_uniform(SEED_BASE + 5, nx) - 1.0)
    recs = [record("e@facet", "e", 0, rec_interval)]
    rho = np.zeros(N)
    rho[2] = 1.0
    return make_problem("qcl-5lvl-comb", L, mats, [(0.0, L, 0)], nx, dt, n_steps, rho,
                        refl=(0.8, 0.8), e_init=e_init, records=recs, precision=precision)


def ladder(N, nx=8192, n_steps=20000, precision=32, rec_interval=100, length=2e-3):
    """Anharmonic N-level ladder (Sec. 4.3): E_1 = 0, E_{n+1} = E_n + hbar w0 (1 - 0.1 (n - 3)),
    w0 = 2 pi 1e13 1/s, any N >= 2 (the paper's level-count benchmark).

    The paper prints only the level energies and the default grid (8192 points, 2 ns);
    the rest is this generator's choice: dipoles on adjacent transitions
    mu_{n,n+1} = 1e-29 sqrt(n) C m (oscillator-like), decay n -> n-1 at 1e10 n 1/s,
    pure dephasing 1e11 1/s on every pair, n3d = 1e24 m^-3, ground state, the medium in the
    middle half of a `length` vacuum domain, a hard Gaussian pulse at w0 (tau 100 fs,
    1e8 V/m) at cell 0, absorbing ends; all populations at the centre and E at 3/4 length
    recorded every `rec_interval` steps.
    """
    c = CODATA
    w0 = 2 * math.pi * 1e13
    en = [0.0]
    for n in range(1, N):
        en.append(en[-1] + c["hbar"] * w0 * (1.0 - 0.1 * (n - 3)))
    mu_off = np.zeros(n_off(N), complex)
    for n in range(1, N):                        # 1-based pair (n, n+1): packed index of (n-1, n)
        i, j = n - 1, n
        mu_off[j * (j - 1) // 2 + i] = 1e-29 * math.sqrt(n)
    rates = np.zeros((N, N))
    for n in range(1, N):
        rates[n - 1, n] = 1e10 * n               # from level n+1 (0-based n) into level n
    deph = np.full(n_off(N), 1e11)
    qm = general_qm(1e24, en, None, None, mu_off, rates, deph)
    mats = [vacuum(), qm_material(qm)]
    regions = [(0.0, 0.25 * length, 0), (0.25 * length, 0.75 * length, 1), (0.75 * length, length, 0)]
    dt = courant_dt(length, nx, c["c0"])
    tau = 100e-15
    src = source("gauss", 0.0, 1e8, w0 / (2 * math.pi), 5.0, 1.0 / tau)
    mid = nx // 2
    recs = [record(f"pop{k}", "pop", mid, rec_interval, i=k, j=k) for k in range(N)]
    recs.append(record("e@3/4", "e", (3 * nx) // 4, rec_interval))
    rho = np.zeros(N)
    rho[0] = 1.0
    return make_problem(f"ladder-{N}lvl", length, mats, regions, nx, dt, n_steps, rho,
                        refl=(0.0, 0.0), sources=[src], records=recs, precision=precision)


def sweep_sim(k, rng, nx=None, n_steps=50000, precision=32, rec_interval=50):
    """One member of the batched parameter sweep (even index: 2 levels, odd: 3)."""
    c = CODATA
    if nx is None:
        nx = int(rng.integers(500, 20001))
    dx = 100e-9
    L = dx * (nx - 1)
    dipole = 1e-29 * rng.uniform(0.5, 2.0)
    n3d = 1e24 * rng.uniform(0.5, 2.0)
    if k % 2 == 0:
        t12 = rng.uniform(0.1e-9, 1e-9)
        qm = two_level_params(n3d, 2 * math.pi * 2e14, dipole / c["e"], 1.0 / t12, 1.0 / t12, -1.0)
        rho = [1.0, 0.0]
        tau = 100e-15 / (2.0 * math.acosh(math.sqrt(2.0)))
        src = source("sech", 0.0, 2.0 * c["hbar"] / (dipole * tau), 2e14, 10.0, 1.0 / tau)
    else:
        qm = _lambda3_material(rng, c)
        qm["n3d"] = n3d
        qm["mu_off"] = qm["mu_off"] * (dipole / 1e-29)
        rho = [0.5, 0.5, 0.0]
        tau = 30e-15
        src = source("gauss", 0.0, math.sqrt(math.pi) * c["hbar"] / (2 * dipole * tau), 190e12,
                     100e-15 / tau, 1.0 / tau)
    mats = [vacuum(), qm_material(qm)]
    regions = [(0.0, 0.1 * L, 0), (0.1 * L, 0.9 * L, 1), (0.9 * L, L, 0)]
    dt = courant_dt(L, nx, c["c0"])
    N = 2 if k % 2 == 0 else 3
    probes = (nx // 3, (2 * nx) // 3)
    recs = []
    for p in probes:
        recs.append(record(f"e@{p}", "e", p, rec_interval))
        for lvl in range(N):
            recs.append(record(f"rho{lvl}{lvl}@{p}", "pop", p, rec_interval, i=lvl, j=lvl))
    return make_problem(f"sweep-{k}", L, mats, regions, nx, dt, n_steps, rho,
                        refl=(0.0, 0.0), sources=[src], records=recs, precision=precision)


def sweep(n_sims=256, n_steps=50000, precision=32, seed=None, nx_range=(500, 20000)):
    """Batched parameter sweep: n_sims independent 2/3-level simulations."""
    rng = np.random.default_rng(SEED_BASE + 3 if seed is None else seed)
    out = []
    for k in range(n_sims):
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        out.append(sweep_sim(k, rng, nx=nx, n_steps=n_steps, precision=precision))
    return out


def serve_trace(n_requests=2000, rate=200.0, seed=None, precision=32,
                nx_range=(1000, 32000), steps_range=(10000, 200000), rec_interval=100):
    """Poisson arrival trace of mixed 2/3/6-level solves for the serving loop.

    Returns a list of (arrival_time_s, problem).  60 % two-level, 30 %
    three-level, 10 % six-level; both ends absorbing; one probe recorded every
    ``rec_interval`` steps.
    """
    rng = np.random.default_rng(SEED_BASE + 4 if seed is None else seed)
    t = 0.0
    out = []
    for k in range(n_requests):
        t += rng.exponential(1.0 / rate)
        u = rng.uniform()
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        nt = int(rng.integers(steps_range[0], steps_range[1] + 1))
        if u < 0.6:
            p = sweep_sim(0, rng, nx=nx, n_steps=nt, precision=precision, rec_interval=rec_interval)
        elif u < 0.9:
            p = sweep_sim(1, rng, nx=nx, n_steps=nt, precision=precision, rec_interval=rec_interval)
        else:
            p = qcl6(nx=nx, n_steps=nt, precision=precision, seed=int(rng.integers(1 << 31)),
                     rec_interval=rec_interval)
            p["refl"] = (0.0, 0.0)
            p["e_init"] = None
            p["sources"] = [source("gauss", 0.0, 1e6, 3e12, 5.0, 1.0 / 500e-15)]
        p["records"] = p["records"][:1]
        p["records"][0]["interval"] = rec_interval
        p["name"] = f"req-{k}"
        out.append((t, p))
    return out


# ---------------------------------------------------------------------------
# Small seeded cases for parity tests
# ---------------------------------------------------------------------------

def random_qm(rng, N, scale_e=None, diag_h0=False, dipole=1e-29):
    """Random Hermitian H0 (energies up to ~1 eV), dipole and Lindblad rates."""
    c = CODATA
    en = np.sort(rng.uniform(0.0, 1.0, N)) * c["e"] * 0.8
    en[0] = 0.0
    h_off = np.zeros(n_off(N), complex)
    if not diag_h0:
        h_off = (rng.normal(size=n_off(N)) + 1j * rng.normal(size=n_off(N))) * 5e-3 * c["e"]
    mu_off = (rng.normal(size=n_off(N)) + 1j * rng.normal(size=n_off(N))) * dipole
    mu_diag = rng.normal(size=N) * 0.2 * dipole
    rates = rng.uniform(0.1e12, 2e12, (N, N))
    np.fill_diagonal(rates, 0.0)
    base = rng.uniform(0.2e12, 1e12)
    u = rng.uniform(0.0, 1e6, N)
    deph = []
    for j in range(1, N):
        for i in range(j):
            deph.append(base + 0.5 * (u[i] - u[j]) ** 2)
    return general_qm(rng.uniform(0.5e24, 2e24), en, h_off, mu_diag, mu_off, rates, deph)


def random_rho(rng, N):
    """A random full-rank density matrix in packed form (diag, off)."""
    a = rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
    rho = a @ a.conj().T
    rho /= np.trace(rho).real
    diag = np.real(np.diag(rho)).copy()
    off = []
    for j in range(1, N):
        for i in range(j):
            off.append(rho[i, j])
    return diag, np.asarray(off, complex)


def random_small(seed, N=3, nx=40, n_steps=60, n_materials=2, refl=(0.0, 1.0),
                 precision=64, vacuum_ends=True, soft=False, e_noise=0.0, rec_interval=1,
                 full_records=True):
    """Tiny random device for brute-force parity: several materials, ragged grid.

    Fields are driven by a strong hard (or soft) sech source so that the
    density matrices move visibly within a few dozen steps.
    """
    c = CODATA
    rng = np.random.default_rng(seed)
    L = 2e-6 * (nx - 1) / 39.0 if nx > 1 else 0.0
    mats = []
    if vacuum_ends:
        mats.append(vacuum(eps_r=rng.uniform(1.0, 2.0)))
    for _ in range(n_materials):
        if N == 0:
            mats.append(vacuum(eps_r=rng.uniform(1.0, 4.0), alpha0=rng.uniform(0, 2e4)))
        else:
            mats.append(qm_material(random_qm(rng, N), eps_r=rng.uniform(1.0, 4.0),
                                    alpha0=rng.uniform(0.0, 2e4), overlap=rng.uniform(0.5, 1.0)))
    regions = []
    if nx > 1:
        cuts = np.sort(rng.uniform(0.1, 0.9, len(mats) - 1)) * L
        edges = np.concatenate([[0.0], cuts, [L]])
        for k in range(len(mats)):
            regions.append((edges[k], edges[k + 1], k))
        eps_min = min(m["eps_r"] * m["mu_r"] for m in mats)
        dt = courant_dt(L, nx, c["c0"] / math.sqrt(eps_min), courant=0.5)
    else:
        regions.append((0.0, 0.0, len(mats) - 1))
        dt = 2e-17
    if N > 0:
        rd, ro = random_rho(rng, N)
    else:
        rd, ro = np.array([1.0]), np.zeros(0, complex)
    width = 1.0 / (rng.uniform(2.0, 6.0) * dt)
    src = source("sech", 0.0, rng.uniform(3e9, 8e9), rng.uniform(1e14, 3e14),
                 4.0, width, phase=rng.uniform(0, 2 * math.pi), hard=not soft)
    srcs = [src]
    if nx > 4:
        srcs.append(source("gauss", node_x(L, nx, nx // 2), rng.uniform(1e9, 3e9), rng.uniform(1e14, 3e14),
                           3.0, 1.0 / (rng.uniform(3.0, 8.0) * dt), hard=False))
    e_init = None
    if e_noise > 0.0:
        e_init = e_noise * (2.0 * splitmix64_uniform(seed, nx) - 1.0)
    recs = []
    if full_records:
        recs.append(record("e", "e", -1, rec_interval))
        recs.append(record("h", "h", -1, rec_interval))
        if N > 0:
            for lvl in range(N):
                recs.append(record(f"rho{lvl}{lvl}", "pop", -1, rec_interval, i=lvl, j=lvl))
            for j in range(1, N):
                for i in range(j):
                    recs.append(record(f"re{i}{j}", "rho_re", -1, rec_interval, i=i, j=j))
                    recs.append(record(f"im{i}{j}", "rho_im", -1, rec_interval, i=i, j=j))
            if N >= 2:
                recs.append(record("inv01", "inv", -1, rec_interval, i=0, j=1))
    return make_problem(f"rand-N{N}-nx{nx}-s{seed}", L, mats, regions, nx, dt, n_steps, rd, ro,
                        refl=refl, e_init=e_init, sources=srcs, records=recs, precision=precision)
