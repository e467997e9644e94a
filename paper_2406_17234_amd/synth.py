"""Seeded synthetic inputs: model atoms, plane-parallel atmospheres, frequency
and angle grids, collision rates.

This module only *draws problem inputs*.  It holds none of the method's
arithmetic (no LTE populations, no profiles, no opacities, no transfer, no
rates); those are computed independently by the HIP library and by the CPU
oracle from what is produced here.  Both sides import this module and nothing
else in common.

Why synthetic: the paper's workloads (Sect. 3.1: the FAL-C atmosphere with 82
depths, Ca II and H I model atoms of Table 1) are not available here, so the
generators below produce inputs of the same shapes: 3-, 6- and 11-level atoms
with overlapping bound-bound and bound-free transitions, energies in [0, 10] eV,
Voigt lines, an isothermal slab and a chromosphere-like temperature rise over a
hydrostatic density stratification, Gauss-Legendre angles on (0, 1) with two
rays per angle (Sect. 2.1.2).

Units are CGS throughout.  Depth index k = 0 is the top of the atmosphere and
z increases downwards (z = -height).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.special import exp1

# CODATA 2018, CGS.  This copy serves the generator only.
H_PLANCK = 6.62607015e-27
C_LIGHT = 2.99792458e10
K_BOLTZ = 1.380649e-16
M_ELECTRON = 9.1093837015e-28
EV = 1.602176634e-12
AMU = 1.66053906660e-24
SIGMA_THOMSON = 6.6524587321e-25
G_SUN = 2.74e4
MU_GAS = 1.3 * AMU  # mean mass per hydrogen atom for the hydrostatic recipe


@dataclass
class Atom:
    """Model atom.  When the atom has bound-free edges its last level is the
    continuum (ground state of the next ion, stage 1) and every edge ends there.

    Transitions are ordered lines first, then bound-free edges; transition t
    connects lower level ``lo[t]`` and upper level ``up[t]``.
    """
    name: str
    E: np.ndarray          # [nlev] level energies, erg, E[0] = 0
    g: np.ndarray          # [nlev] statistical weights
    stage: np.ndarray      # [nlev] int32 ionisation stage: 0 bound, 1 continuum
    line_lo: np.ndarray    # [nline] int32
    line_up: np.ndarray    # [nline] int32
    A_ul: np.ndarray       # [nline] Einstein A, s^-1
    a_damp: np.ndarray     # [nline] Voigt damping parameter (constant)
    mass_amu: float        # atomic mass for the Doppler width
    vturb: float           # microturbulence, cm/s
    bf_lo: np.ndarray      # [nbf] int32 (upper level is always the continuum)
    bf_alpha0: np.ndarray  # [nbf] cross-section at the edge, cm^2 (recipe parameter)

    @property
    def nlev(self):
        return len(self.E)

    @property
    def nline(self):
        return len(self.line_lo)

    @property
    def nbf(self):
        return len(self.bf_lo)

    @property
    def ntr(self):
        return self.nline + self.nbf

    def tr_lo(self):
        return np.concatenate([self.line_lo, self.bf_lo]).astype(np.int32)

    def tr_up(self):
        return np.concatenate([self.line_up,
                               np.full(self.nbf, self.nlev - 1)]).astype(np.int32)

    def line_nu0(self):
        return (self.E[self.line_up] - self.E[self.line_lo]) / H_PLANCK

    def edge_nu0(self):
        return (self.E[-1] - self.E[self.bf_lo]) / H_PLANCK


@dataclass
class Atmos:
    z: np.ndarray        # [nz] cm, increasing downwards
    T: np.ndarray        # [nz] K
    ne: np.ndarray       # [nz] cm^-3
    nH: np.ndarray       # [nz] cm^-3
    ntot: np.ndarray     # [nz] cm^-3, total density of the active atom
    chi_c: np.ndarray    # [nz] gray background opacity, cm^-1
    chi_sca: np.ndarray  # [nz] background scattering opacity, cm^-1 (zeros = none)
    eta_c: np.ndarray | None = None  # [nz, nnu] thermal background emissivity (None: chi_c B_nu)
    vlos: np.ndarray | None = None   # [nz] vertical velocity, cm/s, positive upwards (None: static)

    @property
    def nz(self):
        return len(self.z)


@dataclass
class Grid:
    nu: np.ndarray       # [nnu] union frequency grid, Hz, strictly increasing
    win_lo: np.ndarray   # [ntr] int32, first union index of each transition window
    win_hi: np.ndarray   # [ntr] int32, one past the last union index
    mu: np.ndarray       # [nmu] Gauss-Legendre nodes on (0, 1)
    w_mu: np.ndarray     # [nmu] weights, sum = 1
    bf_nu: list = field(default_factory=list)     # per edge: its own tabulation grid
    bf_alpha: list = field(default_factory=list)  # per edge: cross-section on bf_nu
    w_nu: np.ndarray | None = None  # [nnu] frequency weights (None: trapezoid per window)

    @property
    def nnu(self):
        return len(self.nu)

    @property
    def nmu(self):
        return len(self.mu)


@dataclass
class Problem:
    """One column: everything the library's column-creation call consumes."""
    name: str
    atom: Atom
    atmos: Atmos
    grid: Grid
    C_up: np.ndarray     # [nz, ntr] upward collisional rate l -> u, s^-1
    seed: int = 0

    @property
    def dims(self):
        a = self.atom
        return dict(nz=self.atmos.nz, nlev=a.nlev, ntr=a.ntr, nline=a.nline,
                    nbf=a.nbf, nnu=self.grid.nnu, nmu=self.grid.nmu)

    def depth_points(self):
        """Formal-solution depth-points per residual call: Nnu * 2Nmu * Nz."""
        return self.grid.nnu * 2 * self.grid.nmu * self.atmos.nz


# ----------------------------------------------------------------------------
# atoms
# ----------------------------------------------------------------------------

def _doppler_rel(T, mass_amu, vturb=0.0):
    return np.sqrt(2.0 * K_BOLTZ * T / (mass_amu * AMU) + vturb ** 2) / C_LIGHT


def make_atom(nlev: int, nline: int, seed: int, name: str | None = None,
              overlap_Tmin: float = 4400.0, q_max: float = 50.0) -> Atom:
    """Seeded atom: ``nlev - 1`` bound levels plus a continuum.

    Energies: E_0 = 0, E_c ~ U[6, 10] eV, other bound levels sorted U[1, E_c-0.5]
    eV with consecutive gaps >= 0.3 eV; g in {2,4,6,8,10}, g_c = 1.  Lines are
    distinct bound pairs always including (0, 1), A_ul log-uniform [1e6, 1e8],
    Voigt damping 1e-3, mass 40 amu.  Every bound level has an edge with
    alpha0 log-uniform [1e-19, 1e-17] cm^2.  For six or more levels at least
    one pair of lines is placed inside each other's window (+-q_max Doppler
    widths at ``overlap_Tmin``) by nudging one upper level.
    """
    rng = np.random.default_rng(seed)
    nb = nlev - 1
    if nline > nb * (nb - 1) // 2:
        raise ValueError("too many lines for the number of bound levels")
    for _attempt in range(1000):
        Ec = rng.uniform(6.0, 10.0)
        if nb > 1:
            Eb = np.sort(rng.uniform(1.0, Ec - 0.5, nb - 1))
            Eb = np.concatenate([[0.0], Eb])
            if np.min(np.diff(Eb)) < 0.3:
                continue
        else:
            Eb = np.array([0.0])
        E_eV = np.concatenate([Eb, [Ec]])
        g = np.concatenate([rng.choice([2, 4, 6, 8, 10], nb), [1]]).astype(float)
        pairs = [(i, j) for i in range(nb) for j in range(i + 1, nb) if (i, j) != (0, 1)]
        pick = [(0, 1)] if nb > 1 else []
        if nline > 1:
            idx = rng.choice(len(pairs), nline - 1, replace=False)
            pick += [pairs[i] for i in sorted(idx)]
        pick = pick[:nline]
        lo = np.array([p[0] for p in pick], dtype=np.int32)
        up = np.array([p[1] for p in pick], dtype=np.int32)
        if nlev >= 6:
            E_eV = _force_overlap(E_eV, lo, up, rng, overlap_Tmin, q_max)
            if E_eV is None:
                continue
        A = 10.0 ** rng.uniform(6.0, 8.0, nline)
        alpha0 = 10.0 ** rng.uniform(-19.0, -17.0, nb)
        stage = np.zeros(nlev, np.int32)
        stage[-1] = 1
        return Atom(name=name or f"atom{nlev}_s{seed}", E=E_eV * EV, g=g, stage=stage,
                    line_lo=lo, line_up=up, A_ul=A,
                    a_damp=np.full(nline, 1e-3), mass_amu=40.0, vturb=0.0,
                    bf_lo=np.arange(nb, dtype=np.int32), bf_alpha0=alpha0)
    raise RuntimeError("could not draw an atom")


def _force_overlap(E_eV, lo, up, rng, Tmin, q_max):
    """Nudge one upper level so two lines sit 0.3 window half-widths apart."""
    nb = len(E_eV) - 1
    rel = 0.3 * q_max * _doppler_rel(Tmin, 40.0)
    order = rng.permutation(len(lo))
    for a in order:
        for b in order:
            if a == b or up[b] in (lo[a], up[a]) or up[b] == 0:
                continue
            nu_a = E_eV[up[a]] - E_eV[lo[a]]
            newE = E_eV[lo[b]] + nu_a * (1.0 + rel)
            E2 = E_eV.copy()
            E2[up[b]] = newE
            Eb = E2[:nb]
            if np.any(np.diff(Eb) < 0.3) or newE >= E2[-1] - 0.5 or newE <= 0.5:
                continue
            return E2
    return None


def count_line_overlaps(grid: Grid, nline: int) -> int:
    """Number of line pairs whose windows share union-grid frequencies."""
    c = 0
    for a in range(nline):
        for b in range(a + 1, nline):
            if grid.win_lo[a] < grid.win_hi[b] and grid.win_lo[b] < grid.win_hi[a]:
                c += 1
    return c


# ----------------------------------------------------------------------------
# atmospheres
# ----------------------------------------------------------------------------

def _hydrogen_ion_fraction(T, nH):
    """LTE hydrogen ionisation fraction from the Saha equation (13.6 eV)."""
    s = (2.0 * np.pi * M_ELECTRON * K_BOLTZ * T / H_PLANCK ** 2) ** 1.5 \
        * np.exp(-13.6 * EV / (K_BOLTZ * T)) / nH
    return 0.5 * (-s + np.sqrt(s * s + 4.0 * s))


def isothermal_slab(nz: int = 64, T: float = 5000.0, nH0: float = 1e17,
                    abund: float = 1e-6, tau_top: float = 1e-6,
                    tau_bot: float = 1e3) -> Atmos:
    """Isothermal exponential slab, depths log-spaced in continuum optical depth."""
    Hs = K_BOLTZ * T / (MU_GAS * G_SUN)
    tau = 10.0 ** np.linspace(np.log10(tau_top), np.log10(tau_bot), nz)
    h = -Hs * np.log(tau)
    nH = nH0 * np.exp(-h / Hs)
    sigma_c = 1.0 / (nH0 * Hs)           # tau_cont(h=0) = 1
    Tz = np.full(nz, T)
    return Atmos(z=-h, T=Tz, ne=1e-4 * nH, nH=nH, ntot=abund * nH,
                 chi_c=sigma_c * nH, chi_sca=np.zeros(nz))


def chromosphere_T(h_km):
    h = np.asarray(h_km, dtype=float)
    lo = 4400.0 + 2000.0 * np.clip((500.0 - h) / 600.0, 0.0, None) ** 1.5
    hi = 4400.0 + 5600.0 * np.clip((h - 500.0) / 1500.0, 0.0, None) ** 2
    return np.where(h < 500.0, lo, hi)


def chromosphere(nz: int = 82, nH0: float = 1e17, abund: float = 1e-6,
                 h_top_km: float = 2000.0, h_bot_km: float = -100.0,
                 perturb_seed: int | None = None, perturb_amp: float = 0.1,
                 thomson: bool = False, h_km: np.ndarray | None = None) -> Atmos:
    """Chromosphere-like column: temperature minimum of 4400 K near 500 km,
    1e4 K at 2000 km, hydrostatic hydrogen density, LTE hydrogen electrons.

    With ``perturb_seed`` the temperature is multiplied by (1 + amp*xi(h)), xi
    a clipped sum of three random sinusoids, and the density re-derived.
    Depths: ``nz`` heights evenly spaced from the top down, or the decreasing
    heights ``h_km`` (then ``nz`` is ignored).
    """
    hf = np.linspace(h_bot_km, h_top_km, 8401)
    Tf = chromosphere_T(hf)
    if perturb_seed is not None:
        rng = np.random.default_rng(perturb_seed)
        xi = np.zeros_like(hf)
        for _ in range(3):
            amp = rng.uniform(0.3, 0.7)
            lam = rng.uniform(200.0, 2000.0)
            ph = rng.uniform(0.0, 2.0 * np.pi)
            xi += amp * np.sin(2.0 * np.pi * hf / lam + ph)
        Tf = Tf * (1.0 + perturb_amp * np.clip(xi, -1.0, 1.0))
    # hydrostatic: d ln(nH T)/dh = -mu g/(k T)
    integrand = MU_GAS * G_SUN / (K_BOLTZ * Tf) * 1e5  # per km
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (integrand[1:] + integrand[:-1]) * np.diff(hf))])
    i0 = np.searchsorted(hf, 0.0)
    cum -= cum[i0]
    T0 = Tf[i0]
    nHf = nH0 * (T0 / Tf) * np.exp(-cum)
    # continuum scale: tau_cont(h = 0) = 1, integrating from the top down
    above = hf >= 0.0
    col = np.trapezoid(nHf[above], hf[above]) * 1e5
    sigma_c = 1.0 / col
    h = np.linspace(h_top_km, h_bot_km, nz) if h_km is None else np.asarray(h_km, dtype=float)
    nz = len(h)
    T = np.interp(h, hf, Tf)
    nH = np.exp(np.interp(h, hf, np.log(nHf)))
    ne = nH * (1e-4 + _hydrogen_ion_fraction(T, nH))
    chi_sca = SIGMA_THOMSON * ne if thomson else np.zeros(nz)
    return Atmos(z=-h * 1e5, T=T, ne=ne, nH=nH, ntot=abund * nH,
                 chi_c=sigma_c * nH, chi_sca=chi_sca)


# ----------------------------------------------------------------------------
# grids and collisions
# ----------------------------------------------------------------------------

def gauss_legendre_01(nmu: int):
    x, w = np.polynomial.legendre.leggauss(nmu)
    return 0.5 * (x + 1.0), 0.5 * w


def make_grid(atom: Atom, atmos: Atmos, n_line_pts, n_bf_pts, nmu: int,
              q_max: float = 50.0, v_max: float = 0.0) -> Grid:
    """Union frequency grid of all transitions' own sub-grids.

    Line sub-grid: odd count, v = q_max * sign(t) t^2 with t uniform on [-1, 1],
    in Doppler widths at the column's minimum temperature; with a velocity
    field of largest speed ``v_max`` (cm/s) also points every quarter Doppler
    width out to v_max / v_D + 3 Doppler widths on both sides of the centre,
    so that the Doppler-shifted cores are resolved.  Edge sub-grid:
    geometric from nu0 (1 + 1e-9) to 3 nu0; the edge's cross-section is
    tabulated there as alpha0 (nu0/nu)^3.  Points closer than 1e-12 relative
    are merged.  A transition's window is the run of union points inside the
    span of its own sub-grid.
    """
    nline, nbf = atom.nline, atom.nbf
    if np.isscalar(n_line_pts):
        n_line_pts = [int(n_line_pts)] * nline
    if np.isscalar(n_bf_pts):
        n_bf_pts = [int(n_bf_pts)] * nbf
    Tmin = float(np.min(atmos.T))
    subs, spans = [], []
    nu0 = atom.line_nu0()
    for t in range(nline):
        npt = int(n_line_pts[t]) | 1
        s = np.linspace(-1.0, 1.0, npt)
        v = q_max * np.sign(s) * s * s
        dnu = nu0[t] * _doppler_rel(Tmin, atom.mass_amu, atom.vturb)
        if v_max > 0.0:
            reach = v_max / (C_LIGHT * _doppler_rel(Tmin, atom.mass_amu, atom.vturb)) + 3.0
            core = np.arange(-np.floor(4.0 * reach), np.floor(4.0 * reach) + 1.0) / 4.0
            v = np.unique(np.concatenate([v, core[np.abs(core) < q_max]]))
        sub = nu0[t] + v * dnu
        subs.append(sub)
        spans.append((sub[0], sub[-1]))
    bf_nu, bf_alpha = [], []
    e0 = atom.edge_nu0()
    for t in range(nbf):
        sub = np.geomspace(e0[t] * (1.0 + 1e-9), 3.0 * e0[t], int(n_bf_pts[t]))
        subs.append(sub)
        spans.append((sub[0], sub[-1]))
        bf_nu.append(sub)
        bf_alpha.append(atom.bf_alpha0[t] * (e0[t] / sub) ** 3)
    allnu = np.sort(np.concatenate(subs))
    keep = np.concatenate([[True], np.diff(allnu) > 1e-12 * allnu[1:]])
    nu = allnu[keep]
    lo = np.empty(nline + nbf, dtype=np.int32)
    hi = np.empty(nline + nbf, dtype=np.int32)
    for t, (a, b) in enumerate(spans):
        lo[t] = np.searchsorted(nu, a * (1.0 - 1e-12), side="left")
        hi[t] = np.searchsorted(nu, b * (1.0 + 1e-12), side="right")
    mu, wmu = gauss_legendre_01(nmu)
    return Grid(nu=nu, win_lo=lo, win_hi=hi, mu=mu, w_mu=wmu,
                bf_nu=bf_nu, bf_alpha=bf_alpha)


def make_collisions(atom: Atom, atmos: Atmos, eps: float = 1e-3) -> np.ndarray:
    """Upward collisional rates C_lu [nz, ntr].

    Lines: C_lu = eps A_ul (g_u/g_l) exp(-h nu0/kT), i.e. a downward rate of
    eps A_ul once the library applies detailed balance.  Edges: eps times the
    photo-ionisation rate of the edge's alpha0 (nu0/nu)^3 cross-section in a
    Wien-approximated Planck field, 8 pi alpha0 nu0^3 E1(h nu0/kT) / c^2.
    """
    T = atmos.T[:, None]
    nu0 = atom.line_nu0()[None, :]
    gl = atom.g[atom.line_lo][None, :]
    gu = atom.g[atom.line_up][None, :]
    Cl = eps * atom.A_ul[None, :] * (gu / gl) * np.exp(-H_PLANCK * nu0 / (K_BOLTZ * T))
    e0 = atom.edge_nu0()[None, :]
    x = H_PLANCK * e0 / (K_BOLTZ * T)
    Rw = 8.0 * np.pi * atom.bf_alpha0[None, :] * e0 ** 3 / C_LIGHT ** 2 * exp1(x)
    Cb = eps * Rw
    return np.ascontiguousarray(np.concatenate([Cl, Cb], axis=1))


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

# Abundances (n_tot / n_H), chosen once per atom so the first line is optically
# thin at the top and thick at the bottom of its column (calibrated offline).
ABUND = {3: 2e-7, 6: 2e-6, 11: 2e-6}


def _split_points(nnu, nline, nbf):
    """Split a frequency budget 5:1 between line and edge points."""
    nl = max(11, int(round(nnu * 5.0 / 6.0 / nline)) | 1)
    nb = max(5, int(round(nnu / 6.0 / nbf)))
    return nl, nb


def slab3(nz: int = 64, nmu: int = 3, seed: int = 1) -> Problem:
    """3-level atom (1 line, 2 edges), isothermal 5000 K slab, 64 depths
    log-spaced in continuum optical depth 1e-6..1e3, 61 line + 2x10 edge
    frequencies, 3 angles x 2 rays."""
    atom = make_atom(3, 1, seed, name="atom3")
    atm = isothermal_slab(nz=nz, abund=ABUND[3])
    grid = make_grid(atom, atm, 61, 10, nmu)
    return Problem("slab3", atom, atm, grid, make_collisions(atom, atm), seed)


def chromo6(nz: int = 82, nmu: int = 5, seed: int = 2, nnu: int = 600,
            thomson: bool = False) -> Problem:
    """6-level atom (5 lines, 5 edges), chromosphere-like column of 82
    depths, ~600 frequencies (5 x 100 line + 5 x 20 edge), 5 angles x 2 rays."""
    atom = make_atom(6, 5, seed, name="atom6")
    atm = chromosphere(nz=nz, abund=ABUND[6], thomson=thomson)
    nl, nb = _split_points(nnu, 5, 5)
    grid = make_grid(atom, atm, nl, nb, nmu)
    return Problem("chromo6", atom, atm, grid, make_collisions(atom, atm), seed)


def velocity_step(h_km, v_jump_kms: float = 5.0, h0_km: float = 1000.0,
                  width_km: float = 50.0):
    """Vertical velocity (cm/s, positive upwards) that rises smoothly by
    v_jump around height h0: a sharp positive gradient at the base of the
    chromosphere (Sect. 3.5)."""
    h = np.asarray(h_km, dtype=float)
    return 1e5 * v_jump_kms * 0.5 * (1.0 + np.tanh((h - h0_km) / width_km))


def optimised_heights(atm_fine: Atmos, h_fine_km, vel_fine, nz: int, v_dopp: float):
    """Depth optimisation extended to velocity gradients (Sect. 3.5): nz
    heights placed at equal steps of the combined change of log continuum
    optical depth, log temperature, log density and velocity along a fine
    model (steps of 0.1 dex, 0.01 dex, 0.1 dex and v_dopp / 5 weigh the
    same; the optical depth counted from chi_c x 1000 km at the top).
    Returns decreasing heights, top and bottom kept."""
    z = atm_fine.z
    tau = np.concatenate([[0.0], np.cumsum(0.5 * (atm_fine.chi_c[1:] + atm_fine.chi_c[:-1]) * np.diff(z))])
    tau += atm_fine.chi_c[0] * 1e8
    d = np.sqrt((np.diff(np.log10(tau)) / 0.1) ** 2 + (np.diff(np.log10(atm_fine.T)) / 0.01) ** 2
                + (np.diff(np.log10(atm_fine.nH)) / 0.1) ** 2 + (np.diff(vel_fine) / (0.2 * v_dopp)) ** 2)
    s = np.concatenate([[0.0], np.cumsum(d)])
    return np.interp(np.linspace(0.0, s[-1], nz), s, h_fine_km)


def chromo6_vel(nz: int = 82, nmu: int = 5, seed: int = 2, nnu: int = 600,
                v_jump_kms: float = 5.0) -> Problem:
    """chromo6's atom in the chromosphere with a velocity step of v_jump
    (upwards above 1000 km), on depths optimised for the gradients and a
    frequency grid that resolves the shifted cores (Sect. 3.5)."""
    atom = make_atom(6, 5, seed, name="atom6")
    h_fine = np.linspace(2000.0, -100.0, 4201)
    fine = chromosphere(abund=ABUND[6], h_km=h_fine)
    v_dopp = C_LIGHT * _doppler_rel(float(np.min(fine.T)), atom.mass_amu, atom.vturb)
    h = optimised_heights(fine, h_fine, velocity_step(h_fine, v_jump_kms), nz, v_dopp)
    atm = chromosphere(abund=ABUND[6], h_km=h)
    atm.vlos = velocity_step(h, v_jump_kms)
    nl, nb = _split_points(nnu, 5, 5)
    grid = make_grid(atom, atm, nl, nb, nmu, v_max=float(np.max(np.abs(atm.vlos))))
    return Problem("chromo6_vel", atom, atm, grid, make_collisions(atom, atm), seed)


def chromo11(nz: int = 256, nmu: int = 8, seed: int = 5) -> Problem:
    """11-level atom (20 lines, 10 edges), chromosphere of 256 depths,
    20 x 180 line + 10 x 40 edge = 4000 frequencies, 8 angles x 2 rays."""
    atom = make_atom(11, 20, seed, name="atom11")
    atm = chromosphere(nz=nz, abund=ABUND[11])
    grid = make_grid(atom, atm, 181, 40, nmu)
    return Problem("chromo11", atom, atm, grid, make_collisions(atom, atm), seed)


_ATOM_CACHE: dict = {}


def _cached_atom(nlev):
    if nlev not in _ATOM_CACHE:
        spec = {3: (1, 1), 6: (5, 2), 11: (20, 5)}[nlev]
        _ATOM_CACHE[nlev] = make_atom(nlev, spec[0], spec[1], name=f"atom{nlev}")
    return _ATOM_CACHE[nlev]


def batch6_column(i: int, nmu: int = 5) -> Problem:
    """Column i of the 4096-column batch: the 6-level chromosphere atom, temperature
    perturbed by +-10%, Nz ~ U{64..160}, Nnu ~ U{400..800}."""
    seed = 3_000_000 + i
    rng = np.random.default_rng(seed)
    nz = int(rng.integers(64, 161))
    nnu = int(rng.integers(400, 801))
    atom = _cached_atom(6)
    atm = chromosphere(nz=nz, abund=ABUND[6], perturb_seed=seed)
    nl, nb = _split_points(nnu, atom.nline, atom.nbf)
    grid = make_grid(atom, atm, nl, nb, nmu)
    return Problem(f"batch6[{i}]", atom, atm, grid, make_collisions(atom, atm), seed)


def batch6_vel_column(i: int, nmu: int = 5, static: bool = False) -> Problem:
    """Column i of a batch with velocity fields: batch6's atom and recipe
    (temperature perturbed +-10%, Nz ~ U{64..160}, Nnu ~ U{400..800} before
    the core points) with an upward velocity step of U[2, 8] km/s,
    U[30, 120] km wide, at U[700, 1400] km, on depths optimised for the
    gradients and a line grid resolving the shifted cores (Sect. 3.5).
    static: the same column (same depths and frequencies) without the
    velocity field."""
    seed = 5_000_000 + i
    rng = np.random.default_rng(seed)
    nz = int(rng.integers(64, 161))
    nnu = int(rng.integers(400, 801))
    vj = float(rng.uniform(2.0, 8.0))
    width = float(rng.uniform(30.0, 120.0))
    h0 = float(rng.uniform(700.0, 1400.0))
    atom = _cached_atom(6)
    h_fine = np.linspace(2000.0, -100.0, 4201)
    fine = chromosphere(abund=ABUND[6], perturb_seed=seed, h_km=h_fine)
    v_dopp = C_LIGHT * _doppler_rel(float(np.min(fine.T)), atom.mass_amu, atom.vturb)
    h = optimised_heights(fine, h_fine, velocity_step(h_fine, vj, h0, width), nz, v_dopp)
    atm = chromosphere(abund=ABUND[6], perturb_seed=seed, h_km=h)
    vel = velocity_step(h, vj, h0, width)
    nl, nb = _split_points(nnu, atom.nline, atom.nbf)
    grid = make_grid(atom, atm, nl, nb, nmu, v_max=float(np.max(np.abs(vel))))
    atm.vlos = None if static else vel
    return Problem(f"batch6_vel[{i}]", atom, atm, grid, make_collisions(atom, atm), seed)


def stream_request(j: int, nz_max: int = 256, nnu_max: int = 2000) -> Problem:
    """Request j of the served stream: atom uniform over 3/6/11 levels,
    Nz ~ U{48..nz_max}, Nnu ~ U{200..nnu_max}, Nmu ~ U{3..8} (defaults: the
    served-stream workload; smaller bounds give quick test cases)."""
    seed = 4_000_000 + j
    rng = np.random.default_rng(seed)
    nlev = int(rng.choice([3, 6, 11]))
    nz = int(rng.integers(48, nz_max + 1))
    nnu = int(rng.integers(200, nnu_max + 1))
    nmu = int(rng.integers(3, 9))
    atom = _cached_atom(nlev)
    atm = chromosphere(nz=nz, abund=ABUND[nlev], perturb_seed=seed)
    nl, nb = _split_points(nnu, atom.nline, atom.nbf)
    grid = make_grid(atom, atm, nl, nb, nmu)
    return Problem(f"stream[{j}]", atom, atm, grid, make_collisions(atom, atm), seed)


def stream_arrivals(duration_s: float, rate: float = 2000.0, seed: int = 4):
    """Poisson arrival times (exponential gaps with the given rate)."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration_s:
            return np.array(out)
        out.append(t)


def tiny(nz: int = 6, nmu: int = 2, seed: int = 7, nline_pts: int = 7,
         nbf_pts: int = 3) -> Problem:
    """A 3-level problem small enough for brute-force Jacobians."""
    atom = make_atom(3, 1, seed, name="atom3tiny")
    atm = isothermal_slab(nz=nz, abund=ABUND[3], tau_top=1e-3, tau_bot=10.0)
    grid = make_grid(atom, atm, nline_pts, nbf_pts, nmu)
    return Problem("tiny", atom, atm, grid, make_collisions(atom, atm), seed)


def two_level(eps_eff: float, pts_per_decade: int = 10, nmu: int = 3, npts: int = 41,
              tau_top: float = 1e-4, tau_bot: float | None = None,
              T: float = 6000.0, a_damp: float = 1e-3) -> Problem:
    """Two-level atom (one line, no edges) in an isothermal slab with no
    background continuum, for the scattering-dominated surface law.

    Collisions give a thermalisation parameter eps_eff = C_ul (1 - e^{-h nu0/kT})
    / (A_ul + C_ul (1 - e^{-h nu0/kT})).  Depths are log-spaced in a nominal
    line-centre optical depth from ``tau_top`` to ``tau_bot``.
    """
    E1 = 2.0 * EV
    atom = Atom(name="two-level", E=np.array([0.0, E1]), g=np.array([2.0, 4.0]),
                stage=np.zeros(2, np.int32), line_lo=np.array([0], np.int32),
                line_up=np.array([1], np.int32), A_ul=np.array([1e7]),
                a_damp=np.array([a_damp]), mass_amu=40.0, vturb=0.0,
                bf_lo=np.zeros(0, np.int32), bf_alpha0=np.zeros(0))
    if tau_bot is None:
        tau_bot = max(100.0 / eps_eff, 10.0 * a_damp / eps_eff ** 2)
    ndec = np.log10(tau_bot / tau_top)
    nz = int(round(pts_per_decade * ndec)) + 1
    tau = 10.0 ** np.linspace(np.log10(tau_top), np.log10(tau_bot), nz)
    nu0 = E1 / H_PLANCK
    dop = nu0 * _doppler_rel(T, 40.0)
    B_lu = (4.0 / 2.0) * 1e7 * C_LIGHT ** 2 / (2.0 * H_PLANCK * nu0 ** 3)
    # nominal line-centre opacity per unit lower-level density (Doppler core)
    kap = H_PLANCK * nu0 / (4.0 * np.pi) * B_lu / (np.sqrt(np.pi) * dop)
    nl = 1e10
    z = tau / (kap * nl)
    nz = len(z)
    x = H_PLANCK * nu0 / (K_BOLTZ * T)
    atm = Atmos(z=z, T=np.full(nz, T), ne=np.full(nz, 1e10),
                nH=np.full(nz, 1e14), ntot=np.full(nz, nl * (1.0 + 2.0 * np.exp(-x))),
                chi_c=np.zeros(nz), chi_sca=np.zeros(nz))
    grid = make_grid(atom, atm, npts, [], nmu)
    # eps_eff -> C_ul; the input is the upward rate C_lu = C_ul (g_u/g_l) e^{-x}
    stim = 1.0 - np.exp(-x)
    C_ul = eps_eff * 1e7 / (stim * (1.0 - eps_eff))
    C = np.zeros((nz, 1))
    C[:, 0] = C_ul * (4.0 / 2.0) * np.exp(-x)
    return Problem(f"two-level eps={eps_eff:g}", atom, atm, grid, C, 0)
