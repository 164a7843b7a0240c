"""Plain FP64 CPU oracle for the 1D Maxwell-Bloch method (test infrastructure).

This module is test infrastructure.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product library never
does, and it shares no code with the HIP path.  Everything here is written
for obviousness, not speed: complex N x N density matrices, the Liouvillian
as an explicit N^2 x N^2 superoperator built by applying its definition to
basis matrices, ``scipy.linalg.expm`` for the propagators and
``numpy.linalg.eigh`` for the field part.

What it computes (paper sections cited per function):

* Maxwell's equations in 1D on the Yee grid, update form of eq:eupdate /
  eq:hupdate with the coefficients a', b', c' (Sec. 3.2) and the loss
  relation alpha0 = sqrt(mu/eps) sigma / 2 (Sec. 3.1.1).
* The master equation eq:master1D with H = H0 - mu E and the relaxation
  superoperator given by scattering rates and pure dephasing rates
  (eq:relax_pop and the dephasing equation, Sec. 3.1.1), or by explicit
  Lindblad operators (eq:lindbladdiss with the coefficient matrix
  diagonalised) when a quantum description lists ``lindblad_ops``.
* Weak coupling in time (Sec. 2.2, Fig. 1): rho lives at t_{n+1/2} at the
  E nodes.  The density step exp(L dt) is approximated by an operator
  splitting (Sec. 2.2, "exact step + operator splitting" family); the
  reading used here is Strang splitting with the field part in the middle:
  rho <- e^{L0 dt/2} [ W (e^{L0 dt/2} rho) W^+ ],  W = exp(+i dt E mu / hbar).
* Polarization current (Sec. 2): dP/dt = n3D tr{mu d(rho)/dt}, evaluated at
  t_{n+1/2} from rho^{n+1/2} with L0 only, because tr{mu [mu, rho]} = 0.
* Loop order of Alg. 1: H and rho (and p) first, then E, then edges,
  sources and records.
* Strong coupling (Sec. 2.2 names it beside the weak coupling above, without a
  formula): rho lives at the times of E.  Reading used here: rho^{n+1} is the
  same Strang step driven by the midpoint field (E^n + E^{n+1})/2, and the
  polarization current of eq:ediscrete is the centred difference
  n3D tr{mu (rho^{n+1} - rho^n)}/dt.  The E update of a quantum cell then
  depends on E^{n+1} through rho^{n+1}; it is solved by fixed-point iteration
  to convergence.  Edges and sources follow as in the weak scheme, and every
  quantum cell's rho^{n+1} is finally taken with its final E^{n+1}.
* Field part by a Cayley approximant (the class name lindblad_reg_cayley of
  Sec. 3.2 names the Cayley form; the paper prints no formula): problems with
  field_step == "cayley" replace W = exp(A), A = i dt E mu / hbar, by the
  Cayley transform W_C = (I - A/2)^{-1} (I + A/2), which is unitary for the
  anti-Hermitian A and agrees with exp(A) to second order.

Readings of points the paper leaves open (also listed in the design notes):
edges with R = 1 are a perfect electric conductor (E = 0), edges with R = 0
are a first-order Mur absorbing boundary, and edges with 0 < R < 1 (the
semi-transparent mirrors of Sec. 2.1, whose mechanism the paper does not
give) are a resistive termination: the edge node's half cell is loaded by an
impedance Z_L = eta (1 - sqrt R)/(1 + sqrt R), eta the wave impedance of the
edge material, whose normal-incidence amplitude reflection (Z_L - eta)/
(Z_L + eta) = -sqrt(R); sources are evaluated at t_{n+1};
a hard source sets E, a soft source adds to it, at the node nearest to its
position (ties to the even node); sech source
s(t) = A sech(w t - shift) sin(2 pi f t + phi) and the Gaussian source
s(t) = A exp(-(w t - shift)^2) sin(2 pi f t + phi); records are taken after
step n when (n+1) is a multiple of the interval.
"""
from __future__ import annotations

import math
import numpy as np
import scipy.linalg as sla

# ---------------------------------------------------------------------------
# Quantum mechanical description (Sec. 3.1.1)
# ---------------------------------------------------------------------------


def unpack_hermitian(diag, off):
    """Hermitian matrix from a real diagonal and the packed upper triangle.

    The upper triangle is packed column by column: (1,2), (1,3), (2,3),
    (1,4), ... (Sec. 3.1.1, qm_operator; the ordering is fixed by the
    dephasing-vector description and the QCL listing).
    """
    n = len(diag)
    a = np.zeros((n, n), complex)
    for i in range(n):
        a[i, i] = diag[i]
    k = 0
    for j in range(1, n):
        for i in range(j):
            a[i, j] = off[k]
            a[j, i] = np.conj(off[k])
            k += 1
    return a


def pair_list(n):
    """Packed (i, j) index pairs, i < j, in the qm_operator ordering."""
    return [(i, j) for j in range(1, n) for i in range(j)]


def two_level_description(qm, consts):
    """The simplified two-level constructor (Sec. 3.1.1, qm_desc_2lvl).

    H0 = hbar w21 / 2 diag(-1, 1), mu = -e z21 sigma_x,
    gamma_12 = gamma1 (1 - w0)/2 (2 -> 1), gamma_21 = gamma1 (1 + w0)/2
    (1 -> 2), pure dephasing gamma_12,p = gamma2 - gamma1/2.
    """
    hbar, e = consts["hbar"], consts["e"]
    h0 = hbar * qm["omega21"] / 2.0 * np.diag([-1.0, 1.0]).astype(complex)
    mu = -e * qm["z21"] * np.array([[0.0, 1.0], [1.0, 0.0]], complex)
    g1, g2, w0 = qm["gamma1"], qm["gamma2"], qm["w0"]
    rates = np.array([[0.0, g1 * (1.0 - w0) / 2.0], [g1 * (1.0 + w0) / 2.0, 0.0]])
    deph = np.array([g2 - g1 / 2.0])
    return h0, mu, rates, deph


def describe(qm, consts):
    """(H0, mu, rates, pure_deph, n3d) as full matrices for a qm dict."""
    if qm["kind"] == "2lvl":
        h0, mu, rates, deph = two_level_description(qm, consts)
    else:
        h0 = unpack_hermitian(qm["h0_diag"], qm["h0_off"])
        mu = unpack_hermitian(qm["mu_diag"], qm["mu_off"])
        rates = np.array(qm["rates"], float)
        deph = np.array(qm["pure_deph"], float)
    return h0, mu, rates, deph, qm["n3d"]


def dissipator(rho, rates, deph):
    """Relaxation superoperator in rate form (eq:relax_pop and the dephasing law).

    d rho_ii = sum_{j != i} gamma_ij rho_jj - rho_ii / tau_i,
        1/tau_j = sum_{i != j} gamma_ij  (trace preservation);
    d rho_ij = -[ (1/tau_i + 1/tau_j)/2 + gamma_ij,p ] rho_ij,  i != j.
    rates[i, j] = gamma_ij is the rate from level j into level i.
    """
    n = rho.shape[0]
    inv_tau = np.array([sum(rates[i, j] for i in range(n) if i != j) for j in range(n)])
    out = np.zeros_like(rho)
    for i in range(n):
        acc = -inv_tau[i] * rho[i, i]
        for j in range(n):
            if j != i:
                acc += rates[i, j] * rho[j, j]
        out[i, i] = acc
    for k, (i, j) in enumerate(pair_list(n)):
        g = 0.5 * (inv_tau[i] + inv_tau[j]) + deph[k]
        out[i, j] = -g * rho[i, j]
        out[j, i] = -g * rho[j, i]
    return out


def free_generator(rho, h0, rates, deph, hbar, ops=None):
    """L0(rho) = -i/hbar [H0, rho] + D(rho)  (eq:master1D without the field); D in rate
    form, or from explicit Lindblad operators when ops is given."""
    d = dissipator(rho, rates, deph) if ops is None else lindblad_dissipator(rho, ops)
    return -1j / hbar * (h0 @ rho - rho @ h0) + d


def field_generator(rho, mu, e_field, hbar):
    """L_E(rho) = -i/hbar [-mu E, rho] = +i E / hbar [mu, rho]."""
    return 1j * e_field / hbar * (mu @ rho - rho @ mu)


def superoperator(fn, n):
    """Matrix of a linear map on N x N matrices acting on row-major vec(rho)."""
    s = np.zeros((n * n, n * n), complex)
    for k in range(n * n):
        basis = np.zeros((n, n), complex)
        basis[k // n, k % n] = 1.0
        s[:, k] = fn(basis).reshape(n * n)
    return s


def lindblad_from_rates(rates, deph):
    """Explicit Lindblad operators equivalent to the rate-form dissipator.

    Jump operators sqrt(gamma_ij) |i><j| for every i != j, and diagonal
    operators sqrt(lambda_k) diag(v_k) from the Gram matrix
    G = -1/2 J D J of the squared distances D_ij = 2 gamma_ij,p
    (J = I - 1 1^T / N).  Returns (ops, min_eig(G)); the dissipator is
    completely positive when min_eig(G) >= 0.
    """
    n = rates.shape[0]
    ops = []
    for i in range(n):
        for j in range(n):
            if i != j and rates[i, j] != 0.0:
                op = np.zeros((n, n), complex)
                op[i, j] = math.sqrt(rates[i, j])
                ops.append(op)
    d = np.zeros((n, n))
    for k, (i, j) in enumerate(pair_list(n)):
        d[i, j] = d[j, i] = 2.0 * deph[k]
    jm = np.eye(n) - np.ones((n, n)) / n
    g = -0.5 * jm @ d @ jm
    lam, vec = np.linalg.eigh(g)
    for k in range(n):
        if lam[k] > 1e-12 * max(1.0, abs(lam).max()):
            ops.append(np.diag(math.sqrt(lam[k]) * vec[:, k]).astype(complex))
    return ops, float(lam.min()) if n > 1 else 0.0


def lindblad_dissipator(rho, ops):
    """D(rho) = sum_k L rho L^+ - 1/2 {L^+ L, rho}  (eq:lindbladdiss, diagonalised C)."""
    out = np.zeros_like(rho)
    for op in ops:
        ld = op.conj().T
        out += op @ rho @ ld - 0.5 * (ld @ op @ rho + rho @ ld @ op)
    return out


def is_completely_positive(deph, n, tol=1e-9):
    """The pure dephasing rates admit a positive semi-definite C (Sec. 3.1.1)."""
    _, lam_min = lindblad_from_rates(np.zeros((n, n)), deph)
    scale = max(1.0, float(np.max(np.abs(deph))) if len(deph) else 1.0)
    return lam_min >= -tol * scale


# ---------------------------------------------------------------------------
# Field part (Sec. 2.2 and Sec. 3.2)
# ---------------------------------------------------------------------------


def fdtd_constants(mat, dt, dx, consts):
    """a', b', c' of eq:eupdate / eq:hupdate; sigma from alpha0 (Sec. 3.1.1)."""
    eps = consts["eps0"] * mat["eps_r"]
    mu = consts["mu0"] * mat["mu_r"]
    sigma = 2.0 * mat["alpha0"] * math.sqrt(eps / mu)
    q = dt * sigma / (2.0 * eps)
    a = (1.0 - q) / (1.0 + q)
    b = (dt / eps) / (1.0 + q)
    c = dt / (dx * mu) if dx > 0 else 0.0
    return a, b, c


def light_speed(mat, consts):
    return 1.0 / math.sqrt(consts["eps0"] * mat["eps_r"] * consts["mu0"] * mat["mu_r"])


def source_value(src, t, n=None):
    """Source value at time t = n dt: sech or Gaussian envelope times a carrier, or the
    n-th sample of a sampled waveform (zero after its end; needs n)."""
    if src["kind"] == "table":
        return float(src["table"][n]) if n < len(src["table"]) else 0.0
    env = 0.0
    for q in range(max(1, src["count"])):
        arg = src["width"] * (t - q * src["period"]) - src["shift"]
        if src["kind"] == "sech":
            env += 1.0 / math.cosh(arg) if abs(arg) < 700 else 0.0
        elif src["kind"] == "gauss":
            env += math.exp(-arg * arg)
        else:
            raise ValueError(src["kind"])
    return src["amp"] * env * math.sin(2.0 * math.pi * src["freq"] * t + src["phase"])


def source_cell(x, dx, nx):
    """E node of a source at position x: round(x/dx) with ties to the even node (the
    paper converts positions to integer grid indices at set-up, Sec. 3.2).  A single-point
    device (nx = 1) has its one node at x = 0."""
    if nx == 1:
        if x != 0.0:
            raise ValueError(f"source at x={x} on a single-point device")
        return 0
    cell = round(x / dx)            # Python rounds halves to even
    if not 0 <= cell <= nx - 1:
        raise ValueError(f"source at x={x} lies outside the grid")
    return int(cell)


def material_index(regions, x, dx):
    """Region lookup: [x_start, x_end) first, then closed intervals, then the right end."""
    for r in regions:
        if r["x_start"] <= x < r["x_end"]:
            return r["material"]
    for r in regions:
        if r["x_start"] <= x <= r["x_end"]:
            return r["material"]
    end = max(r["x_end"] for r in regions)
    if end < x <= end + 0.5 * dx:
        return max(regions, key=lambda r: r["x_end"])["material"]
    raise ValueError(f"grid point x={x} lies in no region")


# ---------------------------------------------------------------------------
# The solver (Alg. 1)
# ---------------------------------------------------------------------------


class Oracle:
    """FP64 reference solve of one problem description (see workloads)."""

    def __init__(self, prob):
        self.p = prob
        c = prob["consts"]
        self.c = c
        nx = prob["nx"]
        if nx == 2:
            raise ValueError("nx must be 1 or at least 3")
        self.nx = nx
        self.dt = prob["dt"]
        self.dx = prob["length"] / (nx - 1) if nx > 1 else 0.0
        mats = prob["materials"]
        self.mat_e = np.array([material_index(prob["regions"], m * self.dx, self.dx) for m in range(nx)])
        self.mat_h = np.array([material_index(prob["regions"], (m + 0.5) * self.dx, self.dx)
                               for m in range(max(nx - 1, 0))], dtype=int)
        # per-node FDTD coefficients
        coef = [fdtd_constants(m, self.dt, self.dx, c) for m in mats]
        self.ca = np.array([coef[k][0] for k in self.mat_e])
        self.cb = np.array([coef[k][1] for k in self.mat_e])
        self.gam = np.array([mats[k]["overlap"] for k in self.mat_e])
        self.ch = np.array([coef[k][2] for k in self.mat_h])
        if nx > 1:
            c_max = max(light_speed(m, c) for m in mats)
            if c_max * self.dt > self.dx * (1 + 1e-12):
                raise ValueError("time step violates the Courant condition")
        # quantum systems, one group of cells per material
        self.groups = []
        n_lv = None
        for k, m in enumerate(mats):
            if m["qm"] is None:
                continue
            cells = np.nonzero(self.mat_e == k)[0]
            if len(cells) == 0:
                continue
            h0, mu, rates, deph, n3d = describe(m["qm"], c)
            n = h0.shape[0]
            assert n_lv in (None, n)
            n_lv = n
            hbar = c["hbar"]
            ops = m["qm"].get("lindblad_ops")
            ops = None if ops is None or len(ops) == 0 else [np.asarray(o, complex) for o in ops]
            l0 = superoperator(lambda r: free_generator(r, h0, rates, deph, hbar, ops), n)
            p_half = sla.expm(l0 * (self.dt / 2.0))
            lam, vec = np.linalg.eigh(mu)
            self.groups.append(dict(cells=cells, n=n, h0=h0, mu=mu, rates=rates, deph=deph,
                                    n3d=n3d, l0=l0, p_half=p_half, lam=lam, vec=vec))
        self.levels = n_lv or 0
        # state
        n = self.levels
        self.e = np.zeros(nx) if prob["e_init"] is None else np.array(prob["e_init"], float)
        self.h = np.zeros(max(nx - 1, 0))
        self.p_cur = np.zeros(nx)
        rho0 = unpack_hermitian(prob["rho_diag"], prob["rho_off"]) if n else None
        for g in self.groups:
            g["rho"] = np.repeat(rho0[None, :, :], len(g["cells"]), axis=0).copy()
        self.src_cell = [source_cell(s["x"], self.dx, nx) for s in prob["sources"]]
        self.step_index = 0
        self._apply_edges_init()
        self._apply_sources(0, init=True)
        self.records = {r["name"]: [] for r in prob["records"]}

    # -- boundary handling --------------------------------------------------
    def _mur_coeff(self, cell):
        cl = light_speed(self.p["materials"][self.mat_e[cell]], self.c)
        return (cl * self.dt - self.dx) / (cl * self.dt + self.dx)

    def _load_coeff(self, cell, refl):
        """Half-cell update of an edge node terminated by Z_L (semi-transparent mirror).

        Ampere's law over the half cell [edge, edge +- dx/2] with the load current
        E/Z_L taken at t_{n+1/2} as the mean of E^n and E^{n+1}:
            eps dx/2 (E^{n+1} - E^n)/dt = +-H_inner^{n+1/2} - (E^{n+1} + E^n)/(2 Z_L),
        so E^{n+1} = g E^n +- d H_inner with a = dt/(eps dx Z_L), g = (1 - a)/(1 + a),
        d = 2 dt/(eps dx)/(1 + a) (+ on the left edge, - on the right)."""
        m = self.p["materials"][self.mat_e[cell]]
        eps = self.c["eps0"] * m["eps_r"]
        mu = self.c["mu0"] * m["mu_r"]
        eta = math.sqrt(mu / eps)
        sr = math.sqrt(refl)
        zl = eta * (1.0 - sr) / (1.0 + sr)
        a = self.dt / (eps * self.dx * zl)
        return (1.0 - a) / (1.0 + a), 2.0 * self.dt / (eps * self.dx) / (1.0 + a)

    def _apply_edges_init(self):
        if self.nx < 2:
            return
        if self.p["refl"][0] == 1.0:
            self.e[0] = 0.0
        if self.p["refl"][1] == 1.0:
            self.e[-1] = 0.0

    def _apply_sources(self, n, init=False):
        for s, cell in zip(self.p["sources"], self.src_cell):
            v = source_value(s, n * self.dt, n)
            if s["hard"]:
                self.e[cell] = v
            elif not init:
                self.e[cell] += v

    # -- density step ---------------------------------------------------------
    def _field_op(self, g, e_cells):
        """Cayley field operator (I - A/2)^{-1} (I + A/2), A = i dt E mu / hbar, for
        problems that ask for field_step "cayley" (the exact form is applied by
        _conjugate without forming W)."""
        n = g["n"]
        a = 1j * self.dt / self.c["hbar"] * e_cells[:, None, None] * g["mu"][None, :, :]
        eye = np.eye(n)[None, :, :]
        return np.linalg.solve(eye - 0.5 * a, eye + 0.5 * a)

    def _conjugate(self, g, rho, e_cells):
        """Field part of the step for each cell: W rho W^+ with W = exp(A), A = i dt E mu
        / hbar (Sec. 2.2; the free part is handled by the splitting around it), or
        with the Cayley approximant of W.

        In the eigenbasis of mu (mu = V diag(lam) V^+) W is diagonal, so
        V^+ (W rho W^+) V has entries e^{i dt E (lam_j - lam_k)/hbar} (V^+ rho V)_jk.
        The conjugation is written as rho plus its change,
            W rho W^+ = rho + V [ (e^{i dt E (lam_j - lam_k)/hbar} - 1) (V^+ rho V)_jk ] V^+,
        so that a zero field (W = I) leaves rho exactly as it is, as the definition
        does, instead of passing it through V V^+ = I up to rounding."""
        if self.p.get("field_step", "exact") == "cayley":
            w = self._field_op(g, e_cells)
            return w @ rho @ np.conj(np.transpose(w, (0, 2, 1)))
        vec, lam = g["vec"], g["lam"]
        vh = vec.conj().T
        rp = vh[None, :, :] @ rho @ vec[None, :, :]
        th = self.dt / self.c["hbar"] * e_cells[:, None, None] * (lam[None, :, None] - lam[None, None, :])
        return rho + vec[None, :, :] @ (np.expm1(1j * th) * rp) @ vh[None, :, :]

    def _strang(self, g, rho, e_cells):
        """e^{L0 dt/2} [ W (e^{L0 dt/2} rho) W^+ ] for each cell (W rho W^+ from _conjugate)."""
        k, n = rho.shape[0], g["n"]
        r = (rho.reshape(k, n * n) @ g["p_half"].T).reshape(k, n, n)
        r = self._conjugate(g, r, e_cells)
        return (r.reshape(k, n * n) @ g["p_half"].T).reshape(k, n, n)

    @staticmethod
    def _tr_mu(g, rho):
        return np.real(np.einsum("ij,kji->k", g["mu"], rho))

    def _density_step(self, g, e_cells):
        """Strang splitting: half free step, field conjugation, half free step."""
        k, n = len(g["cells"]), g["n"]
        rho = g["rho"]
        v = rho.reshape(k, n * n) @ g["p_half"].T
        rho = v.reshape(k, n, n)
        # rho <- W rho W^+ (W = exp(i dt E mu / hbar) or its Cayley approximant)
        rho = self._conjugate(g, rho, e_cells)
        v = rho.reshape(k, n * n) @ g["p_half"].T
        g["rho"] = v.reshape(k, n, n)
        # polarization current n3D tr{mu L0(rho)}
        lr = (g["rho"].reshape(k, n * n) @ g["l0"].T).reshape(k, n, n)
        pol = g["n3d"] * np.real(np.einsum("ij,kji->k", g["mu"], lr))
        return pol

    def step(self):
        """One time step n -> n+1 in the order of Alg. 1."""
        if self.p.get("coupling", "weak") == "strong":
            self._step_strong()
            return
        nx, n = self.nx, self.step_index
        e_old = self.e.copy()
        if nx > 1:
            self.h += self.ch * (e_old[1:] - e_old[:-1])
        self.p_cur[:] = 0.0
        for g in self.groups:
            self.p_cur[g["cells"]] = self._density_step(g, e_old[g["cells"]])
        if nx > 1:
            m = slice(1, nx - 1)
            self.e[m] = (self.ca[m] * e_old[m] - self.cb[m] * self.gam[m] * self.p_cur[m]
                         + self.cb[m] / self.dx * (self.h[1:] - self.h[:-1]))
            self._edges(e_old)
        self._apply_sources(n + 1)
        self.step_index = n + 1
        self._record(n)

    def _edges(self, e_old):
        nx = self.nx
        for side, cell, nb in ((0, 0, 1), (1, nx - 1, nx - 2)):
            r = self.p["refl"][side]
            if r == 1.0:
                self.e[cell] = 0.0
            elif r == 0.0:
                kap = self._mur_coeff(cell)
                self.e[cell] = e_old[nb] + kap * (self.e[nb] - e_old[cell])
            elif 0.0 < r < 1.0:
                g, d = self._load_coeff(cell, r)
                h_in = self.h[0] if side == 0 else -self.h[-1]
                self.e[cell] = g * e_old[cell] + d * h_in
            else:
                raise ValueError("reflectivity outside [0, 1]")

    def _step_strong(self):
        """Strong coupling: rho^n, E^n -> rho^{n+1}, E^{n+1} (rho at the times of E)."""
        nx, n = self.nx, self.step_index
        e_old = self.e.copy()
        if nx > 1:
            self.h += self.ch * (e_old[1:] - e_old[:-1])
            m = slice(1, nx - 1)
            e_free = e_old.copy()
            e_free[m] = self.ca[m] * e_old[m] + self.cb[m] / self.dx * (self.h[1:] - self.h[:-1])
            self.e = e_free.copy()
            for g in self.groups:
                cells = g["cells"][(g["cells"] >= 1) & (g["cells"] <= nx - 2)]
                if len(cells) == 0:
                    continue
                sel = np.isin(g["cells"], cells)
                rho_n = g["rho"][sel]
                q_n = self._tr_mu(g, rho_n)
                e_star = e_free[cells].copy()
                for _ in range(100):
                    rho_new = self._strang(g, rho_n, 0.5 * (e_old[cells] + e_star))
                    pol = g["n3d"] * (self._tr_mu(g, rho_new) - q_n) / self.dt
                    e_new = e_free[cells] - self.cb[cells] * self.gam[cells] * pol
                    done = np.max(np.abs(e_new - e_star)) <= 1e-15 * max(1.0, np.max(np.abs(e_new)))
                    e_star = e_new
                    if done:
                        break
                else:
                    raise RuntimeError("strong-coupling field iteration did not converge")
                self.e[cells] = e_star
            self._edges(e_old)
        else:
            self.e = e_old.copy()
        self._apply_sources(n + 1)
        self.p_cur[:] = 0.0
        for g in self.groups:
            rho_n = g["rho"]
            g["rho"] = self._strang(g, rho_n, 0.5 * (e_old[g["cells"]] + self.e[g["cells"]]))
            self.p_cur[g["cells"]] = g["n3d"] * (self._tr_mu(g, g["rho"]) - self._tr_mu(g, rho_n)) / self.dt
        self.step_index = n + 1
        self._record(n)

    # -- observables ----------------------------------------------------------
    def density_at(self, cell):
        for g in self.groups:
            hit = np.nonzero(g["cells"] == cell)[0]
            if len(hit):
                return g["rho"][hit[0]]
        return None

    def _density_value(self, rec, cell):
        rho = self.density_at(cell)
        if rho is None:
            return 0.0
        q, i, j = rec["quantity"], rec["i"], rec["j"]
        if q == "pop":
            return rho[i, i].real
        if q == "inv":
            return (rho[j, j] - rho[i, i]).real
        if q == "rho_re":
            return rho[i, j].real
        if q == "rho_im":
            return rho[i, j].imag
        raise ValueError(q)

    def _value(self, rec, cell):
        if rec["quantity"] == "e":
            return self.e[cell]
        if rec["quantity"] == "h":
            return self.h[cell] if cell < self.nx - 1 else 0.0
        return self._density_value(rec, cell)

    def _record(self, n):
        for r in self.p["records"]:
            if (n + 1) % r["interval"] != 0:
                continue
            if r["cell"] >= 0:
                self.records[r["name"]].append(self._value(r, r["cell"]))
            else:
                self.records[r["name"]].append([self._value(r, m) for m in range(self.nx)])

    def run(self, n_steps=None):
        n_steps = self.p["n_steps"] if n_steps is None else n_steps
        for _ in range(n_steps):
            self.step()
        return {k: np.array(v) for k, v in self.records.items()}

    def full_density(self):
        """(nx, N, N) density matrices; identity/N placeholders outside quantum cells."""
        n = self.levels
        out = np.zeros((self.nx, n, n), complex)
        for g in self.groups:
            out[g["cells"]] = g["rho"]
        return out


def run(prob, n_steps=None):
    """Convenience: records of a full oracle run as a dict name -> array."""
    return Oracle(prob).run(n_steps)
