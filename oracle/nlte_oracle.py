"""FP64 CPU oracle for the residual F(n) of multilevel NLTE statistical
equilibrium and for the Jacobian-free Newton-Krylov (JFNK) solve built on it.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this module; only the test-suite, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP library: the only
common import is the seeded input generator, which contains none of the
method's arithmetic.

Every function follows the paper (Arramy, de la Cruz Rodriguez & Leenaarts,
"Jacobian-free Newton-Krylov method for multilevel NLTE radiative transfer
problems"); docstrings cite the section, equation, algorithm or appendix.
Plain NumPy in float64 (complex128 where the complex-step Jacobian needs it),
vectorised over frequency and angle with a Python loop over depth.

Readings of points the paper leaves open are listed in the design notes; the
ones that change numbers here are:
  * rate normalisation carries the 4 pi of the solid-angle integral (so the
    spontaneous rate of a line at zero intensity equals A_ul);
  * frequency quadrature: trapezoid weights over each transition's own window
    on the union grid; line profiles renormalised per depth on that window;
  * the conservation row replaces the most populated level (lowest index on
    ties); Jacobian-vector products keep the rows of the Newton iterate;
  * piecewise-linear coefficients use their Taylor series below dtau = 0.1;
  * preconditioner "first solution" (background-scattering derivative dropped),
    with |mu| in the ingoing-ray coefficients;
  * convergence on the scaled residual |F| / (gross rate in + out).
"""
from __future__ import annotations

import math
from types import SimpleNamespace

import numpy as np
from scipy.special import wofz

# CODATA 2018 CGS constants (the oracle's own copy)
HP = 6.62607015e-27
CL = 2.99792458e10
KB = 1.380649e-16
ME = 9.1093837015e-28
AMU_G = 1.66053906660e-24
SQRT_PI = math.sqrt(math.pi)


# ----------------------------------------------------------------------------
# setup: n-independent quantities (Sect. 2.1.1)
# ----------------------------------------------------------------------------

def planck(nu, T):
    """Planck function B_nu(T) (boundary condition of Sect. 2.1.2)."""
    return 2.0 * HP * nu ** 3 / CL ** 2 / np.expm1(HP * nu / (KB * T))


def lte_populations(E, g, stage, T, ne, ntot):
    """Saha-Boltzmann populations n*, Sect. 2.1.1 (the Saha-Boltzmann function
    Phi_ij and the LTE ratio in the b-f g_ij).  Returns [nz, nlev] with
    sum_i n*_i = n_tot."""
    T = np.asarray(T)[:, None]
    ne = np.asarray(ne)[:, None]
    lnw = np.log(g)[None, :] - E[None, :] / (KB * T)
    saha = np.log(2.0 * (2.0 * np.pi * ME * KB * T / HP ** 2) ** 1.5 / ne)
    lnw = lnw + stage[None, :] * saha
    lnw -= lnw.max(axis=1, keepdims=True)
    w = np.exp(lnw)
    return np.asarray(ntot)[:, None] * w / w.sum(axis=1, keepdims=True)


def voigt_H(a, v):
    """Voigt function H(a, v) = Re w(v + i a) (line profiles, Sect. 3.1)."""
    return wofz(v + 1j * a).real


def window_weights(nu_win):
    """Trapezoid weights over one transition's window (quadrature coefficients
    omega_nu of Sect. 2.1.2; used unless the grid brings its own weights)."""
    w = np.empty_like(nu_win)
    d = np.diff(nu_win)
    w[0] = 0.5 * d[0]
    w[-1] = 0.5 * d[-1]
    w[1:-1] = 0.5 * (d[1:] + d[:-1])
    return w


def setup(prob):
    """Build the tables that do not depend on the populations: LTE n*,
    Planck B, background emissivity (the atmosphere's eta_c if it has one,
    else chi_c B_nu), the unified transition coefficients V_ij and g_ij
    (Sect. 2.1.1) on each transition window, collision rates in both
    directions (detailed balance), quadrature weights (the grid's w_nu over
    each window if it has them, else trapezoid weights per window)."""
    a, atm, gr = prob.atom, prob.atmos, prob.grid
    nz, nlev, ntr, nline = atm.nz, a.nlev, a.ntr, a.nline
    nu = gr.nu
    T = atm.T
    nstar = lte_populations(a.E, a.g, a.stage, T, atm.ne, atm.ntot)
    B = planck(nu[None, :], T[:, None])                  # [nz, nnu]
    lo = a.tr_lo()
    up = a.tr_up()
    tr = []
    w_nu = getattr(gr, "w_nu", None)
    vel = getattr(atm, "vlos", None)
    vel = None if vel is None else np.asarray(vel, dtype=float)
    for t in range(ntr):
        f0, f1 = int(gr.win_lo[t]), int(gr.win_hi[t])
        nuw = nu[f0:f1]
        w = window_weights(nuw) if w_nu is None else np.array(w_nu[f0:f1], dtype=float)
        c = 4.0 * np.pi * w / (HP * nuw)                  # 4 pi w / (h nu)
        l, u = int(lo[t]), int(up[t])
        if t < nline:
            nu0 = (a.E[u] - a.E[l]) / HP
            B_ul = a.A_ul[t] * CL ** 2 / (2.0 * HP * nu0 ** 3)
            B_lu = a.g[u] / a.g[l] * B_ul
            dnuD = nu0 / CL * np.sqrt(2.0 * KB * T / (a.mass_amu * AMU_G) + a.vturb ** 2)
            v = (nuw[None, :] - nu0) / dnuD[:, None]
            phi = voigt_H(a.a_damp[t], v) / (SQRT_PI * dnuD[:, None])
            phi = phi / (phi * w[None, :]).sum(axis=1, keepdims=True)
            V = HP * nuw[None, :] / (4.0 * np.pi) * B_lu * phi
            gt = np.full((nz, f1 - f0), a.g[l] / a.g[u])
            extra = dict(phi=phi, B_lu=B_lu, nu0=nu0)
            if vel is not None:
                # the profile each ray sees, Doppler-shifted by the velocity
                # component along it (Sect. 3.5): centre nu0 (1 + s v / c)
                # with s = +mu for the outgoing and -mu for the ingoing ray of
                # an angle; normalised per (ray, depth) on the window
                phir = np.empty((2 * gr.nmu, nz, f1 - f0))
                for r in range(2 * gr.nmu):
                    sgn = 1.0 if r < gr.nmu else -1.0
                    proj = sgn * gr.mu[r % gr.nmu] * vel
                    vr = (nuw[None, :] - nu0 * (1.0 + proj[:, None] / CL)) / dnuD[:, None]
                    pr = voigt_H(a.a_damp[t], vr) / (SQRT_PI * dnuD[:, None])
                    phir[r] = pr / (pr * w[None, :]).sum(axis=1, keepdims=True)
                extra.update(phir=phir, Vr=HP * nuw[None, None, :] / (4.0 * np.pi) * B_lu * phir)
        else:
            e = t - nline
            alpha = np.interp(nuw, gr.bf_nu[e], gr.bf_alpha[e])
            V = np.broadcast_to(alpha[None, :], (nz, f1 - f0)).copy()
            ratio = nstar[:, l] / nstar[:, u]
            gt = ratio[:, None] * np.exp(-HP * nuw[None, :] / (KB * T[:, None]))
            extra = {}
        tr.append(SimpleNamespace(t=t, lo=l, up=u, f0=f0, f1=f1, nu=nuw, w=w, c=c,
                                  V=V, g=gt, is_line=t < nline, **extra))
    C_lu = prob.C_up.copy()
    C_ul = C_lu * nstar[:, lo] / nstar[:, up]
    chi_c = np.broadcast_to(atm.chi_c[:, None], (nz, gr.nnu)).copy()
    eta_given = getattr(atm, "eta_c", None)
    eta_c = chi_c * B if eta_given is None else np.array(eta_given, dtype=float)
    dz = np.abs(np.diff(atm.z))
    return SimpleNamespace(prob=prob, nz=nz, nlev=nlev, ntr=ntr, nline=nline,
                           nnu=gr.nnu, nmu=gr.nmu, nu=nu, T=T, nstar=nstar, B=B,
                           tr=tr, lo=lo, up=up, C_lu=C_lu, C_ul=C_ul,
                           chi_c=chi_c, eta_c=eta_c, chi_sca=atm.chi_sca.copy(),
                           ntot=atm.ntot.copy(), z=atm.z.copy(), dz=dz,
                           mu=gr.mu.copy(), w_mu=gr.w_mu.copy(),
                           two_h_nu3_c2=2.0 * HP * nu ** 3 / CL ** 2,
                           vel=vel is not None, nray=2 * gr.nmu)


# ----------------------------------------------------------------------------
# formal solution (Sect. 2.1.2, Appendix A.1)
# ----------------------------------------------------------------------------

_SERIES_DTAU = 0.1
_SERIES_TERMS = 14


def ab_coefficients(dtau):
    """e = exp(-dtau) and the piecewise-linear coefficients a, b of
    Appendix A.1:  a = 1 - (1 - e)/dtau,  b = (1 - e)/dtau - e.

    Below dtau = 0.1 both use their Taylor series (the same functions expanded
    about 0) to avoid the cancellation in 1 - (1 - e)/dtau.  Accepts complex
    dtau (complex-step Jacobians); the branch follows the real part.
    """
    dtau = np.asarray(dtau)
    e = np.exp(-dtau)
    with np.errstate(divide="ignore", invalid="ignore"):
        omx = -np.expm1(-dtau)
        t1 = omx / dtau
        a = 1.0 - t1
        b = t1 - e
    small = np.real(dtau) < _SERIES_DTAU
    if np.any(small):
        x = dtau[small]
        sa = np.zeros_like(x)
        sb = np.zeros_like(x)
        # a = sum_{m>=1} (-1)^{m+1} x^m/(m+1)!, b = sum_{m>=1} (-1)^{m+1} m x^m/(m+1)!
        for m in range(_SERIES_TERMS, 0, -1):
            cm = (-1.0) ** (m + 1) / math.factorial(m + 1)
            sa = sa + cm
            sb = sb + cm * m
            if m > 1:
                sa = sa * x
                sb = sb * x
        a = np.array(a, copy=True)
        b = np.array(b, copy=True)
        a[small] = sa * x
        b[small] = sb * x
    return e, a, b


def formal_solution(chi, S, z, mu, I_bottom, want_coeffs=False):
    """Short-characteristics piecewise-linear formal solution (Eqs. Iplus and
    Iminus, Sect. 2.1.2; boundary conditions I+ = B at the bottom, I- = 0 at
    the top).

    chi, S: [nz, nnu]; mu: [nmu] in (0, 1); I_bottom: [nnu].
    Returns I+ and I- as [nz, nnu, nmu] (and per-segment e, a, b, dtau of
    shape [nz-1, nnu, nmu] when ``want_coeffs``).
    """
    nz = chi.shape[0]
    dz = np.abs(np.diff(z))
    dt = np.result_type(chi, S, float)
    dtau = dz[:, None, None] * (chi[:-1, :, None] + chi[1:, :, None]) / (2.0 * mu[None, None, :])
    e, a, b = ab_coefficients(dtau)
    Ip = np.empty((nz,) + chi.shape[1:] + (len(mu),), dtype=dt)
    Im = np.empty_like(Ip)
    Ip[-1] = I_bottom[:, None]
    for k in range(nz - 2, -1, -1):
        Ip[k] = Ip[k + 1] * e[k] + a[k] * S[k][:, None] + b[k] * S[k + 1][:, None]
    Im[0] = 0.0
    for k in range(1, nz):
        Im[k] = Im[k - 1] * e[k - 1] + a[k - 1] * S[k][:, None] + b[k - 1] * S[k - 1][:, None]
    if want_coeffs:
        return Ip, Im, (e, a, b, dtau)
    return Ip, Im


# ----------------------------------------------------------------------------
# residual F(n)  (Algorithm 1, Eqs. chi, eta, Rij, Rji, residuals)
# ----------------------------------------------------------------------------

def opacity(tb, n, Jdag):
    """Total opacity and emissivity, Eqs. chi and eta of Sect. 2.1.1.
    n: [nz, nlev]; Jdag: [nz, nnu] lagged mean intensity for the background
    scattering term.  Returns chi, eta as [nz, nnu]."""
    dt = np.result_type(n, float)
    chi = (tb.chi_c + tb.chi_sca[:, None]).astype(dt)
    eta = (tb.eta_c + tb.chi_sca[:, None] * Jdag).astype(dt)
    for tr in tb.tr:
        nl = n[:, tr.lo][:, None]
        nu_ = n[:, tr.up][:, None]
        chi[:, tr.f0:tr.f1] += tr.V * (nl - tr.g * nu_)
        eta[:, tr.f0:tr.f1] += tb.two_h_nu3_c2[None, tr.f0:tr.f1] * tr.g * tr.V * nu_
    return chi, eta


def rates_from_J(tb, J):
    """Radiative rate coefficients R_lu, R_ul [nz, ntr] (Eqs. Rij, Rji with the
    4 pi of the solid-angle integral; static atmosphere, so V does not depend
    on mu and the angle integral reduces to the mean intensity J)."""
    dt = np.result_type(J, float)
    R_lu = np.zeros((tb.nz, tb.ntr), dtype=dt)
    R_ul = np.zeros((tb.nz, tb.ntr), dtype=dt)
    for tr in tb.tr:
        Jw = J[:, tr.f0:tr.f1]
        cV = tr.c[None, :] * tr.V
        R_lu[:, tr.t] = (cV * Jw).sum(axis=1)
        R_ul[:, tr.t] = (cV * tr.g * (tb.two_h_nu3_c2[None, tr.f0:tr.f1] + Jw)).sum(axis=1)
    return R_lu, R_ul


def mean_line_intensity(tb, J):
    """Profile-weighted mean intensity Jbar_t = sum_f w_f phi_t J of each line."""
    out = np.zeros((tb.nz, tb.nline), dtype=np.result_type(J, float))
    for tr in tb.tr[:tb.nline]:
        out[:, tr.t] = (tr.w[None, :] * tr.phi * J[:, tr.f0:tr.f1]).sum(axis=1)
    return out


def conservation_rows(n):
    """Level replaced by particle conservation at each depth: the most
    populated one (Algorithm 1, last loop); ties go to the lowest index."""
    return np.argmax(np.real(n), axis=1)


def assemble_F(tb, n, R_lu, R_ul, rows):
    """Rate-equation residual rows and conservation rows (Eqs. residuals_1,
    residuals_2; Algorithm 1 second half).  Also returns the gross rate
    G_i = sum_p n_i(C_ip+R_ip) + n_p(C_pi+R_pi) (n_tot on conservation rows)."""
    dt = np.result_type(n, R_lu, float)
    F = np.zeros((tb.nz, tb.nlev), dtype=dt)
    G = np.zeros((tb.nz, tb.nlev), dtype=float)
    for t in range(tb.ntr):
        l, u = tb.lo[t], tb.up[t]
        out_l = n[:, l] * (tb.C_lu[:, t] + R_lu[:, t])
        out_u = n[:, u] * (tb.C_ul[:, t] + R_ul[:, t])
        kappa = out_l - out_u
        F[:, l] += kappa
        F[:, u] -= kappa
        gross = np.abs(np.real(out_l)) + np.abs(np.real(out_u))
        G[:, l] += gross
        G[:, u] += gross
    k = np.arange(tb.nz)
    F[k, rows] = tb.ntot - n.sum(axis=1)
    G[k, rows] = tb.ntot
    return F, G


def residual(tb, n, Jdag=None, rows=None, want_P=False, I_override=None):
    """Residual vector F(n) of Algorithm 1.

    n: [nz, nlev] (real or complex for complex-step derivatives);
    Jdag: lagged mean intensity [nz, nnu] for the scattering emissivity
    (default B_nu(T)); rows: conservation rows (default: most populated level
    of n); want_P: also build the block-Jacobi preconditioner; I_override:
    replace the formal solution by a given isotropic intensity field [nz, nnu]
    (used to test the rate equations on their own).  With a velocity field
    (Sect. 3.5) the opacity, the formal solution and the line rates are taken
    ray by ray (residual_rays).
    Returns a namespace with F, rho (scaled residual), J, R_lu, R_ul, Jbar,
    rows and optionally P [nz, nlev, nlev].
    """
    if Jdag is None:
        Jdag = tb.B
    if rows is None:
        rows = conservation_rows(n)
    if tb.vel:
        return residual_rays(tb, n, Jdag, rows, want_P, I_override)
    chi, eta = opacity(tb, n, Jdag)
    S = eta / chi
    if I_override is None:
        Ip, Im, co = formal_solution(chi, S, tb.z, tb.mu, tb.B[-1], want_coeffs=True)
        J = (0.5 * tb.w_mu[None, None, :] * (Ip + Im)).sum(axis=2)
    else:
        J = I_override
        Ip = Im = co = None
    R_lu, R_ul = rates_from_J(tb, J)
    F, G = assemble_F(tb, n, R_lu, R_ul, rows)
    out = SimpleNamespace(F=F, G=G, rho=np.abs(F) / G, J=J, R_lu=R_lu, R_ul=R_ul,
                          Jbar=mean_line_intensity(tb, J), rows=rows,
                          chi=chi, S=S)
    if want_P:
        out.P = preconditioner(tb, n, R_lu, R_ul, rows, chi, S, Ip, Im, co)
    return out


# ----------------------------------------------------------------------------
# atmospheres with a velocity field (Sect. 3.5): opacity per ray
# ----------------------------------------------------------------------------

def ray_weights(tb):
    """Angle weight w_m / 2 of each ray: rays 0..nmu-1 outgoing (+mu_m),
    nmu..2 nmu-1 ingoing (-mu_m)."""
    return np.concatenate([0.5 * tb.w_mu, 0.5 * tb.w_mu])


def opacity_rays(tb, n, Jdag):
    """Eqs. chi and eta for every ray: the lines use the profile the ray sees
    (Doppler-shifted by the velocity along it); the background and the
    bound-free terms do not depend on the ray.  [nray, nz, nnu] each."""
    dt = np.result_type(n, float)
    chi0 = (tb.chi_c + tb.chi_sca[:, None]).astype(dt)
    eta0 = (tb.eta_c + tb.chi_sca[:, None] * Jdag).astype(dt)
    for tr in tb.tr[tb.nline:]:
        nl = n[:, tr.lo][:, None]
        nu_ = n[:, tr.up][:, None]
        chi0[:, tr.f0:tr.f1] += tr.V * (nl - tr.g * nu_)
        eta0[:, tr.f0:tr.f1] += tb.two_h_nu3_c2[None, tr.f0:tr.f1] * tr.g * tr.V * nu_
    chi = np.repeat(chi0[None], tb.nray, axis=0)
    eta = np.repeat(eta0[None], tb.nray, axis=0)
    for tr in tb.tr[:tb.nline]:
        nl = n[:, tr.lo][None, :, None]
        nu_ = n[:, tr.up][None, :, None]
        chi[:, :, tr.f0:tr.f1] += tr.Vr * (nl - tr.g[None] * nu_)
        eta[:, :, tr.f0:tr.f1] += tb.two_h_nu3_c2[None, None, tr.f0:tr.f1] * tr.g[None] * tr.Vr * nu_
    return chi, eta


def formal_rays(tb, chi, S):
    """The formal solution of Eqs. Iplus/Iminus along every ray with that
    ray's own opacity and source function.  Returns I [nray, nz, nnu] and the
    segment coefficients of each ray."""
    I = np.empty(chi.shape, dtype=np.result_type(chi, S, float))
    co = []
    for r in range(tb.nray):
        m = r % tb.nmu
        Ip, Im, c = formal_solution(chi[r], S[r], tb.z, tb.mu[m:m + 1], tb.B[-1], want_coeffs=True)
        I[r] = (Ip if r < tb.nmu else Im)[:, :, 0]
        co.append((Ip, Im, c))
    return I, co


def residual_rays(tb, n, Jdag, rows, want_P, I_override=None):
    """F(n) of Algorithm 1 with a velocity field: the rates (Eqs. Rij, Rji)
    keep their angle integral, sum over rays of (w_m/2) V_ray I_ray, since V
    depends on the ray; J (background scattering, outputs) and the
    profile-averaged intensity Jbar are the same angle sums.  I_override
    [nz, nnu]: the intensity of every ray (no formal solution, no P)."""
    chi, eta = opacity_rays(tb, n, Jdag)
    S = eta / chi
    if I_override is None:
        I, co = formal_rays(tb, chi, S)
    else:
        if want_P:
            raise ValueError("want_P needs the formal solution")
        I = np.repeat(np.asarray(I_override)[None], tb.nray, axis=0)
        co = None
    wr = ray_weights(tb)
    J = (wr[:, None, None] * I).sum(axis=0)
    dt = np.result_type(J, float)
    R_lu = np.zeros((tb.nz, tb.ntr), dtype=dt)
    R_ul = np.zeros((tb.nz, tb.ntr), dtype=dt)
    Jbar = np.zeros((tb.nz, tb.nline), dtype=dt)
    for tr in tb.tr:
        Iw = I[:, :, tr.f0:tr.f1]
        if tr.is_line:
            VI = (wr[:, None, None] * tr.Vr * Iw).sum(axis=0)
            Vbar = (wr[:, None, None] * tr.Vr).sum(axis=0)
            R_lu[:, tr.t] = (tr.c[None, :] * VI).sum(axis=1)
            R_ul[:, tr.t] = (tr.c[None, :] * tr.g *
                             (tb.two_h_nu3_c2[None, tr.f0:tr.f1] * Vbar + VI)).sum(axis=1)
            Jbar[:, tr.t] = (tr.w[None, :] * (wr[:, None, None] * tr.phir * Iw).sum(axis=0)).sum(axis=1)
        else:
            Jw = J[:, tr.f0:tr.f1]
            cV = tr.c[None, :] * tr.V
            R_lu[:, tr.t] = (cV * Jw).sum(axis=1)
            R_ul[:, tr.t] = (cV * tr.g * (tb.two_h_nu3_c2[None, tr.f0:tr.f1] + Jw)).sum(axis=1)
    F, G = assemble_F(tb, n, R_lu, R_ul, rows)
    out = SimpleNamespace(F=F, G=G, rho=np.abs(F) / G, J=J, R_lu=R_lu, R_ul=R_ul, Jbar=Jbar,
                          rows=rows, chi=chi, S=S, I=I)
    if want_P:
        out.P = preconditioner_rays(tb, n, R_lu, R_ul, rows, chi, S, co)
    return out


def preconditioner_rays(tb, n, R_lu, R_ul, rows, chi, S, co):
    """The diagonal blocks of Sect. 2.5.1/2.5.2 (first solution) with a
    velocity field: the local derivative of each ray's intensity (App. A.2,
    with that ray's chi and S) times the ray's own alpha, beta, gamma."""
    nz, L = tb.nz, tb.nlev
    P = np.zeros((nz, L, L), dtype=np.result_type(n, float))
    for t in range(tb.ntr):
        l, u = tb.lo[t], tb.up[t]
        r_lu = tb.C_lu[:, t] + R_lu[:, t]
        r_ul = tb.C_ul[:, t] + R_ul[:, t]
        P[:, l, l] += r_lu
        P[:, u, u] += r_ul
        P[:, l, u] -= r_ul
        P[:, u, l] -= r_lu
    wr = ray_weights(tb)
    for r in range(tb.nray):
        m = r % tb.nmu
        Ip, Im, c = co[r]
        a_chi, a_eta, c_chi, c_eta = intensity_derivatives(chi[r], S[r], Ip, Im, c, tb.dz,
                                                           tb.mu[m:m + 1])
        if r < tb.nmu:
            Dchi, Deta = a_chi[:, :, 0], a_eta[:, :, 0]
        else:
            Dchi, Deta = c_chi[:, :, 0], c_eta[:, :, 0]
        alpha, beta, gamma = level_coefficients(tb, n, ray=r)
        X = beta * Dchi[:, :, None] + gamma * Deta[:, :, None]
        P += wr[r] * np.einsum("kfi,kfj->kij", alpha, X)
    k = np.arange(nz)
    P[k, rows, :] = -1.0
    return P


# ----------------------------------------------------------------------------
# block-Jacobi preconditioner (Sect. 2.5.2 "first solution", Appendix A.2)
# ----------------------------------------------------------------------------

def intensity_derivatives(chi, S, Ip, Im, co, dz, mu):
    """Local derivatives of I with respect to chi and eta at the same depth
    (Appendix A.2): a_chi, a_eta for outgoing rays (zero at the bottom where
    I+ is prescribed) and c_chi, c_eta for ingoing rays (zero at the top),
    with |mu| in both.  Returns D_chi = sum_m (w_m/2)(a_chi + c_chi) style
    sums are formed by the caller; here arrays [nz, nnu, nmu]."""
    e, a, b, dtau = co
    nz = chi.shape[0]
    Sx = S[:, :, None]
    Cx = chi[:, :, None]
    h = dz[:, None, None] / (2.0 * mu[None, None, :])
    a_chi = np.zeros_like(Ip)
    a_eta = np.zeros_like(Ip)
    c_chi = np.zeros_like(Ip)
    c_eta = np.zeros_like(Ip)
    # outgoing: depth k uses segment k (k, k+1), k = 0..nz-2
    common = h * (e * (Sx[1:] - Ip[1:]) - (Sx[1:] - Sx[:-1]) * b / dtau)
    a_chi[:-1] = -(Sx[:-1] / Cx[:-1]) * a + common
    a_eta[:-1] = a / Cx[:-1]
    # ingoing: depth k uses segment k-1 (k-1, k), k = 1..nz-1
    common_m = h * (e * (Sx[:-1] - Im[:-1]) - (Sx[:-1] - Sx[1:]) * b / dtau)
    c_chi[1:] = -(Sx[1:] / Cx[1:]) * a + common_m
    c_eta[1:] = a / Cx[1:]
    return a_chi, a_eta, c_chi, c_eta


def level_coefficients(tb, n, ray=None):
    """alpha_i (times the rate quadrature weight), beta_j = d chi / d n_j and
    gamma_j = d eta / d n_j of Sect. 2.5.1, each [nz, nnu, nlev]; with a
    velocity field, those of one ray (its line profiles)."""
    dt = np.result_type(n, float)
    shape = (tb.nz, tb.nnu, tb.nlev)
    alpha = np.zeros(shape, dtype=dt)
    beta = np.zeros(shape)
    gamma = np.zeros(shape)
    for tr in tb.tr:
        sl = slice(tr.f0, tr.f1)
        V = tr.Vr[ray] if (ray is not None and tr.is_line) else tr.V
        A = V * (n[:, tr.lo][:, None] - tr.g * n[:, tr.up][:, None])
        cA = tr.c[None, :] * A
        alpha[:, sl, tr.lo] += cA
        alpha[:, sl, tr.up] -= cA
        beta[:, sl, tr.lo] += V
        beta[:, sl, tr.up] -= tr.g * V
        gamma[:, sl, tr.up] += tb.two_h_nu3_c2[None, sl] * tr.g * V
    return alpha, beta, gamma


def preconditioner(tb, n, R_lu, R_ul, rows, chi, S, Ip, Im, co):
    """Diagonal blocks P^k of the Jacobian (Sect. 2.5.1, 2.5.2 first solution):
    P^k = Gamma^k + sum_nu alpha_i (beta_j D_chi + gamma_j D_eta), with
    D_chi, D_eta the angle-averaged local intensity derivatives, and the
    conservation row replaced by -1 (derivative of n_tot - sum n)."""
    nz, L = tb.nz, tb.nlev
    P = np.zeros((nz, L, L), dtype=np.result_type(n, float))
    # Gamma_ij = delta_ij sum_p (C_ip + R_ip) - (C_ji + R_ji)
    for t in range(tb.ntr):
        l, u = tb.lo[t], tb.up[t]
        r_lu = tb.C_lu[:, t] + R_lu[:, t]
        r_ul = tb.C_ul[:, t] + R_ul[:, t]
        P[:, l, l] += r_lu
        P[:, u, u] += r_ul
        P[:, l, u] -= r_ul
        P[:, u, l] -= r_lu
    a_chi, a_eta, c_chi, c_eta = intensity_derivatives(chi, S, Ip, Im, co, tb.dz, tb.mu)
    wm = 0.5 * tb.w_mu[None, None, :]
    Dchi = (wm * (a_chi + c_chi)).sum(axis=2)
    Deta = (wm * (a_eta + c_eta)).sum(axis=2)
    alpha, beta, gamma = level_coefficients(tb, n)
    X = beta * Dchi[:, :, None] + gamma * Deta[:, :, None]
    P += np.einsum("kfi,kfj->kij", alpha, X)
    k = np.arange(nz)
    P[k, rows, :] = -1.0
    return P


def lu_factor_blocks(P):
    """LU factors (partial pivoting) of every per-depth block."""
    import scipy.linalg as sla
    return [sla.lu_factor(P[k]) for k in range(P.shape[0])]


def lu_solve_blocks(lus, x):
    import scipy.linalg as sla
    out = np.empty_like(x)
    for k, lu in enumerate(lus):
        out[k] = sla.lu_solve(lu, x[k])
    return out


# ----------------------------------------------------------------------------
# Jacobian-vector products and brute-force Jacobians (Sect. 2.4.1-2.4.2)
# ----------------------------------------------------------------------------

def jvp_fd(tb, n, v, F0, eps, Jdag=None, rows=None):
    """Forward-difference product (F(n + eps v) - F(n)) / eps (Eq. fordif),
    with the conservation rows and lagged J held at those of n."""
    if rows is None:
        rows = conservation_rows(n)
    Fp = residual(tb, n + eps * v, Jdag=Jdag, rows=rows).F
    return (Fp - F0) / eps


def jvp_complex_step(tb, n, v, Jdag=None, rows=None, h=1e-200):
    """Complex-step product Im F(n + i h v) / h (Eq. complex, Sect. 2.4.2),
    with the conservation rows and lagged J held at those of n.  No
    subtraction of nearby values takes place, so the step can be as small as
    the paper's 1e-200: the result is the directional derivative of F to
    rounding, linear in v."""
    if rows is None:
        rows = conservation_rows(n)
    Fc = residual(tb, np.asarray(n, float) + 1j * h * np.asarray(v, float), Jdag=Jdag, rows=rows).F
    return Fc.imag / h


def jacobian_complex_step(tb, n, Jdag=None, rows=None, h=1e-20):
    """Dense Jacobian by the complex-step scheme (Eq. complex), one column per
    population: Im F(n + i h e_j) / h.  For tiny grids only."""
    if rows is None:
        rows = conservation_rows(n)
    N = n.size
    Jm = np.empty((N, N))
    for j in range(N):
        dn = np.zeros(N, dtype=complex)
        dn[j] = 1j * h
        Fc = residual(tb, n.astype(complex) + dn.reshape(n.shape), Jdag=Jdag, rows=rows).F
        Jm[:, j] = Fc.imag.ravel() / h
    return Jm


# ----------------------------------------------------------------------------
# Krylov solver (Sect. 2.3): left-preconditioned restarted GMRES
# ----------------------------------------------------------------------------

def gmres(matvec, b, rtol=1e-3, m=30, maxit=200, x0=None):
    """GMRES(m) (Arnoldi with modified Gram-Schmidt and one
    re-orthogonalisation, Givens rotations) from the initial guess x0 (zero
    by default; Algorithm 2 also names -P^-1 f); stops when
    ||b - A x|| <= rtol ||b||.  Returns (x, products with A, final relative
    residual); a nonzero x0 costs one product for r0 = b - A x0."""
    N = b.size
    x = np.zeros(N)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, 0.0
    r = b.copy()
    it = 0
    if x0 is not None:
        x = np.array(x0, dtype=float)
        r = b - matvec(x)
        it = 1
    rel = 1.0
    while it < maxit:
        beta = np.linalg.norm(r)
        V = np.zeros((m + 1, N))
        Hm = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            w = matvec(V[j])
            it += 1
            for _ in range(2):
                for i in range(j + 1):
                    hij = V[i] @ w
                    Hm[i, j] += hij
                    w = w - hij * V[i]
            Hm[j + 1, j] = np.linalg.norm(w)
            if Hm[j + 1, j] > 0:
                V[j + 1] = w / Hm[j + 1, j]
            for i in range(j):
                tmp = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                Hm[i + 1, j] = -sn[i] * Hm[i, j] + cs[i] * Hm[i + 1, j]
                Hm[i, j] = tmp
            den = math.hypot(Hm[j, j], Hm[j + 1, j])
            cs[j] = Hm[j, j] / den
            sn[j] = Hm[j + 1, j] / den
            Hm[j, j] = den
            Hm[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            j_done = j + 1
            rel = abs(g[j + 1]) / bnorm
            if rel <= rtol or it >= maxit:
                break
        y = np.linalg.solve(np.triu(Hm[:j_done, :j_done]), g[:j_done])
        x = x + V[:j_done].T @ y
        if rel <= rtol or it >= maxit:
            break
        r = b - matvec_restart(matvec, x)
    return x, it, rel


def matvec_restart(matvec, x):
    return matvec(x)


# ----------------------------------------------------------------------------
# Krylov solver (Sect. 2.3): BiCGSTAB, the paper's second inner solver
# ----------------------------------------------------------------------------

def bicgstab(matvec, b, rtol=1e-3, maxit=200, x0=None):
    """BiCGSTAB (van der Vorst 1992, as cited in Sect. 2.3): Lanczos-type
    bi-orthogonal directions with a one-parameter minimal-residual smoothing
    step, two products with A per iteration.  Initial guess x0 (zero by
    default; a nonzero one costs one product for r0 = b - A x0), shadow
    residual r^ = r0; stops when ||r|| <= rtol ||b|| (checked on the
    half-step residual s and on r), on a breakdown (rho or (r^, v) or omega
    zero), or after maxit products.  Returns (x, products, final relative
    residual)."""
    N = b.size
    x = np.zeros(N)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, 0.0
    r = b.copy()
    products = 0
    if x0 is not None:
        x = np.array(x0, dtype=float)
        r = b - matvec(x)
        products = 1
    rh = r.copy()
    p = r.copy()
    rho = rh @ r
    rel = 1.0
    while products < maxit:
        v = matvec(p)
        products += 1
        den = rh @ v
        if den == 0.0 or rho == 0.0:
            break
        alpha = rho / den
        s_ = r - alpha * v
        rel = np.linalg.norm(s_) / bnorm
        if rel <= rtol or products >= maxit:
            x = x + alpha * p
            break
        t = matvec(s_)
        products += 1
        tt = t @ t
        omega = (t @ s_) / tt if tt > 0.0 else 0.0
        x = x + alpha * p + omega * s_
        r = s_ - omega * t
        rel = np.linalg.norm(r) / bnorm
        if rel <= rtol or omega == 0.0:
            break
        rho_new = rh @ r
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        rho = rho_new
    return x, products, rel


# ----------------------------------------------------------------------------
# Newton driver (Sect. 2.2, Algorithm 2)
# ----------------------------------------------------------------------------

def zero_radiation_guess(tb):
    """Radiation-free populations (Sect. 2.2.1): per depth, the rate equations
    with J = 0 (spontaneous emission kept) plus particle conservation on the
    most populated level of the result (re-solved if that level changes)."""
    R_lu, R_ul = rates_from_J(tb, np.zeros((tb.nz, tb.nnu)))
    n = np.empty((tb.nz, tb.nlev))
    rows0 = conservation_rows(tb.nstar)
    for k in range(tb.nz):
        M0 = np.zeros((tb.nlev, tb.nlev))
        for t in range(tb.ntr):
            l, u = tb.lo[t], tb.up[t]
            r_lu = tb.C_lu[k, t] + R_lu[k, t]
            r_ul = tb.C_ul[k, t] + R_ul[k, t]
            M0[l, l] += r_lu
            M0[u, u] += r_ul
            M0[l, u] -= r_ul
            M0[u, l] -= r_lu
        row = rows0[k]
        for _ in range(tb.nlev):
            M = M0.copy()
            M[row, :] = 1.0
            rhs = np.zeros(tb.nlev)
            rhs[row] = tb.ntot[k]
            n[k] = np.linalg.solve(M, rhs)
            new = int(np.argmax(n[k]))
            if new == row:
                break
            row = new
    return n


def fd_step(N, vnorm, eps_mach=2.0 ** -52):
    """Difference step eps_2 of Fig. 2 (r = 2) for the scaled unknowns, whose
    population vector is all ones: sqrt(eps_mach) sqrt(1 + sqrt(N)) / ||v||."""
    return math.sqrt(eps_mach) * math.sqrt(1.0 + math.sqrt(N)) / vnorm


def positivity_limit(n, dn, factor=3.0):
    """Per-depth limit of the Newton correction (Sect. 2.2.2, which limits the
    correction at each depth independently and leaves the form open): the
    factor lambda_k <= 1 of depth k keeps every level of n + lambda_k dn
    within [n / factor, factor n], i.e. lambda_k = min(1,
    (1 - 1/factor) min_{dn_i<0} n_i/|dn_i|, (factor - 1) min_{dn_i>0} n_i/dn_i).
    Positive populations stay positive, and no level moves by more than the
    factor in one step."""
    with np.errstate(divide="ignore", invalid="ignore"):
        r_neg = np.where(dn < 0.0, n / -dn, np.inf)
        r_pos = np.where(dn > 0.0, n / dn, np.inf)
    lam = np.minimum(1.0, (1.0 - 1.0 / factor) * r_neg.min(axis=1))
    return np.minimum(lam, (factor - 1.0) * r_pos.min(axis=1))


def solve(tb, n0=None, init="lte", ftol=1e-8, rtol=1e-3, maxiter=50, m=30,
          max_krylov=200, max_halvings=8, Jdag0=None, eps_mach=2.0 ** -52,
          verbose=False, krylov="gmres", jv="fd", krylov_x0="zero"):
    """JFNK solve of F(n) = 0 (Algorithm 2) with left block-Jacobi
    preconditioning, populations scaled by the Newton iterate for the
    finite-difference product, per-depth positivity limiting and damped
    backtracking (Sect. 2.2.2).  The backtracking compares the norm the Krylov
    step reduces, ||D^-1 P^-1 F||_2 with the iterate's P, D and conservation
    rows held fixed, and asks for an Armijo decrease (1 - 1e-4 alpha).
    Convergence: ||rho||_inf <= ftol.  krylov: "gmres" (GMRES(m)) or
    "bicgstab" (max_krylov then counts products with the Jacobian).
    jv: "fd" (forward difference, Eq. fordif) or "complex" (complex step,
    Eq. complex) for the Jacobian-vector products.  krylov_x0: "zero" or
    "precond" (x0 = -P^-1 F, the second initial guess of Algorithm 2, which in
    the scaled unknowns is b itself).

    Lagged scattering term (Sect. 2.1.1, Algorithm 2 "update J"): F(n0) uses
    the initial estimate Jdag0 (default B_nu(T)).  At every accepted Newton
    point J-dagger becomes the J of that point's evaluation; when the
    atmosphere has background scattering, F is then evaluated again at the
    same point with the new J-dagger, so that F(n), the Krylov products and
    the line search of the next Newton step all see one J-dagger (the
    difference of Eq. fordif would otherwise pick up the change of J-dagger
    between its two terms).

    A line search that ends on a non-finite merit (every trial failed, the
    last one overflowed) stops the solve with status "nonfinite".

    Returns a namespace with n, J (the J-dagger of the final F: with it,
    F(n; J) is the residual the stopping test saw; without scattering F does
    not depend on it and it is the J of the final evaluation), history and
    call counts (one call per formal solution; re-assigning conservation rows
    at an accepted point repeats no formal solution and is not counted).
    """
    if n0 is None:
        n0 = tb.nstar.copy() if init == "lte" else zero_radiation_guess(tb)
    n = np.array(n0, dtype=float)
    Jdag = tb.B.copy() if Jdag0 is None else np.array(Jdag0, dtype=float)
    has_sca = bool(np.any(tb.chi_sca != 0.0))
    res = residual(tb, n, Jdag=Jdag, want_P=True)
    calls = 1
    hist = [dict(rho=res.rho.max(), Finf=np.abs(res.F).max(), dn=np.nan, krylov=0)]
    converged = res.rho.max() <= ftol
    it = 0
    stalls = 0
    status = None
    N = n.size
    while not converged and it < maxiter:
        rows = res.rows
        lus = lu_factor_blocks(res.P)
        D = n.copy()
        F0 = res.F

        def matvec(u):
            nonlocal calls
            un = np.linalg.norm(u)
            if un == 0.0:
                return np.zeros_like(u)
            if jv == "complex":
                Jv = jvp_complex_step(tb, n, D * u.reshape(n.shape), Jdag=Jdag, rows=rows)
            else:
                eps = fd_step(N, un, eps_mach)
                Jv = jvp_fd(tb, n, D * u.reshape(n.shape), F0, eps, Jdag=Jdag, rows=rows)
            calls += 1
            return (lu_solve_blocks(lus, Jv) / D).ravel()

        b = -(lu_solve_blocks(lus, F0) / D).ravel()
        phi0 = np.linalg.norm(b)
        x0 = b.copy() if krylov_x0 == "precond" and phi0 > 0.0 else None
        if krylov == "bicgstab":
            u, kit, krel = bicgstab(matvec, b, rtol=rtol, maxit=max_krylov, x0=x0)
        else:
            u, kit, krel = gmres(matvec, b, rtol=rtol, m=m, maxit=max_krylov, x0=x0)
        dn = D * u.reshape(n.shape)
        lam = positivity_limit(n, dn)[:, None]
        alpha = 1.0
        for h in range(max_halvings + 1):
            trial = n + alpha * lam * dn
            rt = residual(tb, trial, Jdag=Jdag, rows=rows)
            calls += 1
            phi = np.linalg.norm(lu_solve_blocks(lus, rt.F) / D)
            if phi < (1.0 - 1e-4 * alpha) * phi0:
                break
            if h == max_halvings:
                stalls += 1
                break
            alpha *= 0.5
        if not np.isfinite(phi):
            # every trial failed and the last one is not even finite (an
            # inverted line turned the opacity negative): stop, n unchanged
            status = "nonfinite"
            break
        n_prev = n
        n = trial
        res = residual(tb, n, Jdag=Jdag, want_P=True)
        Jdag = res.J
        if has_sca:
            res = residual(tb, n, Jdag=Jdag, want_P=True)
            calls += 1
        it += 1
        dnorm = 0.5 * np.max(np.abs((n - n_prev) / (n + n_prev)))
        hist.append(dict(rho=res.rho.max(), Finf=np.abs(res.F).max(), dn=dnorm,
                         krylov=kit, krel=krel, alpha=alpha))
        if verbose:
            print(f"newton {it}: rho={res.rho.max():.3e} dn={dnorm:.3e} "
                  f"krylov={kit} alpha={alpha}")
        converged = res.rho.max() <= ftol
    if status is None:
        status = "converged" if converged else "maxiter"
    return SimpleNamespace(n=n, J=Jdag, res=res, iters=it, calls=calls,
                           converged=converged, history=hist, stalls=stalls, status=status)


def dense_newton(tb, n0, ftol=1e-12, maxiter=30, verbose=False):
    """Plain Newton-Raphson with the complex-step Jacobian (tiny grids only),
    used to cross-check the JFNK root."""
    n = np.array(n0, dtype=float)
    for it in range(maxiter):
        res = residual(tb, n)
        if res.rho.max() <= ftol:
            return n, it
        Jm = jacobian_complex_step(tb, n, rows=res.rows)
        dn = np.linalg.solve(Jm, -res.F.ravel()).reshape(n.shape)
        lam = positivity_limit(n, dn)[:, None]
        n = n + lam * dn
        if verbose:
            print(it, res.rho.max())
    return n, maxiter
