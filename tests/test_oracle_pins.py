"""Pins of the CPU oracle against facts fixed by the paper and by mathematics:
closed forms, identities, special cases and brute force on tiny grids.

Each test names the part of the oracle it pins and the passage it follows.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

from oracle import nlte_oracle as O
from paper_2406_17234_amd import synth as S


# ---------------------------------------------------------------- formal solver

def _closed_form_linear(z, chi0, s0, s1, mu, Ib):
    """Exact solutions of Eqs. RTE1/RTE2 for constant opacity and a source
    function linear in vertical optical depth, S = s0 + s1 tau."""
    tau = chi0 * (z - z[0])
    T = tau[-1]
    St = s0 + s1 * tau
    ST = s0 + s1 * T
    Ip = St + mu * s1 - (ST + mu * s1 - Ib) * np.exp(-(T - tau) / mu)
    Im = St - mu * s1 - (s0 - mu * s1) * np.exp(-tau / mu)
    return Ip, Im


@pytest.mark.parametrize("mu", [0.05, 0.3, 0.9])
def test_formal_solution_exact_for_linear_source(mu):
    """Eqs. Iplus/Iminus (piecewise-linear short characteristics) reproduce the
    exact intensity when S is linear in tau and chi is constant, for optically
    thin (series branch) and thick (direct branch) steps alike."""
    rng = np.random.default_rng(3)
    steps = np.concatenate([10 ** rng.uniform(-5, -2, 40), 10 ** rng.uniform(-1.5, 1.0, 40)])
    rng.shuffle(steps)
    chi0 = 2.0
    z = np.concatenate([[0.0], np.cumsum(steps / chi0)])
    s0, s1, Ib = 3.0, 0.7, 9.0
    tau = chi0 * z
    chi = np.full((len(z), 1), chi0)
    Sv = (s0 + s1 * tau)[:, None]
    Ip, Im = O.formal_solution(chi, Sv, z, np.array([mu]), np.array([Ib]))
    Ipx, Imx = _closed_form_linear(z, chi0, s0, s1, mu, Ib)
    assert np.max(np.abs(Ip[:, 0, 0] / Ipx - 1)) < 1e-13
    # I- starts at exactly zero; compare relative where it is not tiny
    m = Imx > 1e-6
    assert np.max(np.abs(Im[m, 0, 0] / Imx[m] - 1)) < 1e-12
    assert np.max(np.abs(Im[:, 0, 0] - Imx)) < 1e-13 * s0


def test_formal_solution_constant_source_linear_opacity():
    """Constant S with chi linear in z: the trapezoid optical-depth step is
    exact, I+ = B everywhere (e + a + b = 1) and I- = B (1 - exp(-tau/mu))."""
    z = np.linspace(0.0, 5.0, 60) ** 1.5
    chi = (0.3 + 2.0 * z)[:, None]
    tau = 0.3 * z + z ** 2
    B = 4.2
    mu = np.array([0.2, 0.7])
    Ip, Im = O.formal_solution(chi, np.full_like(chi, B), z, mu, np.array([B]))
    assert np.max(np.abs(Ip - B)) < 1e-13 * B
    exact = B * (1.0 - np.exp(-tau[:, None] / mu[None, :]))
    assert np.max(np.abs(Im[:, 0, :] - exact)) < 1e-13 * B


def test_ab_coefficients_against_high_precision():
    """Appendix A.1 coefficients a, b against 40-digit decimal arithmetic on
    both sides of the series switch, plus a + b = 1 - e and 0 <= a, b <= 1."""
    getcontext().prec = 40
    x = np.array([1e-9, 1e-6, 1e-3, 0.03, 0.0999, 0.1, 0.1001, 0.5, 3.0, 30.0, 700.0])
    e, a, b = O.ab_coefficients(x)
    for xi, ai, bi, ei in zip(x, a, b, e):
        X = Decimal(repr(float(xi)))
        E = (-X).exp()
        A = 1 - (1 - E) / X
        Bc = (1 - E) / X - E
        assert abs(float(Decimal(repr(float(ai))) / A - 1)) < 4e-15
        assert abs(float(Decimal(repr(float(bi))) / Bc - 1)) < 4e-15
        assert abs(float(Decimal(repr(float(ei))) / E - 1)) < 4e-16 or float(E) < 1e-300
    assert np.all((a >= 0) & (a <= 1) & (b >= 0) & (b <= 1))
    assert np.allclose(a + b, -np.expm1(-x), rtol=1e-15, atol=0)


# --------------------------------------------------------------- setup tables

def test_planck_identity():
    """(2 h nu^3/c^2 + B_nu) exp(-h nu/kT) = B_nu, the identity behind
    detailed balance of Eqs. Rij/Rji at J = B."""
    nu = np.geomspace(1e13, 3e16, 50)[None, :]
    T = np.array([3000.0, 6000.0, 2e4])[:, None]
    B = O.planck(nu, T)
    lhs = (2 * O.HP * nu ** 3 / O.CL ** 2 + B) * np.exp(-O.HP * nu / (O.KB * T))
    assert np.max(np.abs(lhs / B - 1)) < 1e-12


def test_saha_textbook_constant():
    """Hydrogen-like Saha ratio from the Saha-Boltzmann function of Sect. 2.1.1
    against the textbook value n_e n_p / n_1 = 2.4147e15 T^1.5 exp(-13.6 eV/kT)
    (g_1 = 2, g_p = 1)."""
    E = np.array([0.0, 13.6 * S.EV])
    g = np.array([2.0, 1.0])
    stage = np.array([0, 1])
    T = np.array([6000.0, 1e4, 2e4])
    ne = np.array([1e11, 1e12, 1e13])
    n = O.lte_populations(E, g, stage, T, ne, np.ones(3))
    ratio = ne * n[:, 1] / n[:, 0]
    ref = 2.4147e15 * T ** 1.5 * np.exp(-13.6 * S.EV / (O.KB * T))
    assert np.max(np.abs(ratio / ref - 1)) < 2e-4
    assert np.allclose(n.sum(axis=1), 1.0, rtol=1e-15)


def test_voigt_special_cases():
    """Voigt function used for the line profiles (Sect. 3.1): H(0, v) = exp(-v^2),
    H(a, 0) = exp(a^2) erfc(a), and its integral over v is sqrt(pi)."""
    from scipy.special import erfc
    v = np.linspace(-6, 6, 101)
    assert np.max(np.abs(O.voigt_H(0.0, v) - np.exp(-v * v))) < 1e-14
    for a in [1e-3, 0.1, 1.0]:
        assert abs(O.voigt_H(a, 0.0) / (np.exp(a * a) * erfc(a)) - 1) < 1e-13
    vv = np.linspace(-2000, 2000, 2_000_001)
    integ = np.trapezoid(O.voigt_H(0.01, vv), vv)
    # tails beyond |v| = 2000 contribute ~ 2 a / (sqrt(pi) 2000)
    assert abs(integ + 2 * 0.01 / 2000 / math.sqrt(math.pi) * math.sqrt(math.pi) - math.sqrt(math.pi)) < 1e-4


def test_window_weights_exact_for_linear():
    """Trapezoid frequency weights integrate linear functions exactly."""
    nu = np.sort(np.random.default_rng(1).uniform(1, 2, 37))
    w = O.window_weights(nu)
    f = 3.0 - 2.0 * nu
    assert abs((w * f).sum() - (3 * (nu[-1] - nu[0]) - (nu[-1] ** 2 - nu[0] ** 2))) < 1e-14


def test_profiles_normalised():
    tb = O.setup(S.chromo6())
    for tr in tb.tr[:tb.nline]:
        assert np.allclose((tr.phi * tr.w[None, :]).sum(axis=1), 1.0, rtol=1e-14)


# ------------------------------------------------------------- opacity, rates

def test_lte_source_function_is_planck():
    """With LTE populations the emissivity-to-opacity ratio of Eqs. chi/eta is
    the Planck function: exact where only bound-free and background terms act,
    to O(h dnu/kT) inside lines (their stimulated term uses g_ij = g_i/g_j)."""
    tb = O.setup(S.chromo6())
    chi, eta = O.opacity(tb, tb.nstar, tb.B)
    Sf = eta / chi
    in_line = np.zeros(tb.nnu, bool)
    for tr in tb.tr[:tb.nline]:
        in_line[tr.f0:tr.f1] = True
    assert np.max(np.abs(Sf[:, ~in_line] / tb.B[:, ~in_line] - 1)) < 1e-13
    assert np.max(np.abs(Sf[:, in_line] / tb.B[:, in_line] - 1)) < 2e-3


def test_spontaneous_rate_equals_einstein_A():
    """At zero intensity the downward rate of a line (Eq. Rji) is the
    spontaneous rate A_ul: pins the 4 pi normalisation and the Einstein
    relations inside V_ij (to the (nu/nu0)^3 spread over the profile)."""
    p = S.chromo6()
    tb = O.setup(p)
    R_lu, R_ul = O.rates_from_J(tb, np.zeros((tb.nz, tb.nnu)))
    assert np.all(R_lu == 0)
    for t in range(tb.nline):
        assert np.max(np.abs(R_ul[:, t] / p.atom.A_ul[t] - 1)) < 1e-5


def _einstein_B_lu(atom, t):
    """Einstein relations (textbook): B_ul = A_ul c^2 / (2 h nu0^3),
    g_l B_lu = g_u B_ul."""
    lo, up = atom.line_lo[t], atom.line_up[t]
    nu0 = (atom.E[up] - atom.E[lo]) / O.HP
    return atom.g[up] / atom.g[lo] * atom.A_ul[t] * O.CL ** 2 / (2 * O.HP * nu0 ** 3), nu0


@pytest.mark.parametrize("maker", [S.chromo6, S.chromo11])
def test_mean_line_intensity_of_a_flat_field(maker):
    """Profile-averaged line intensity Jbar_t = sum_f w_f phi_t J (the
    absorption-profile average behind Eq. Rij): a field that does not vary
    with frequency is returned unchanged at every depth, because each profile
    is normalised on its own window with the same weights."""
    tb = O.setup(maker())
    c = np.geomspace(1e-3, 1e3, tb.nz)[:, None]
    Jb = O.mean_line_intensity(tb, c * np.ones((1, tb.nnu)))
    assert Jb.shape == (tb.nz, tb.nline)
    assert np.max(np.abs(Jb / c - 1)) < 1e-14


def test_upward_line_rate_is_B_lu_times_mean_line_intensity():
    """Eq. Rij with V_ij = (h nu / 4 pi) B_lu phi (Sect. 2.1.1) and the 4 pi of
    the solid angle: R_lu = B_lu Jbar_t for any radiation field, with B_lu
    from the Einstein relations."""
    p = S.chromo6()
    tb = O.setup(p)
    rng = np.random.default_rng(4)
    J = tb.B * np.exp(rng.standard_normal(tb.B.shape))
    R_lu, _ = O.rates_from_J(tb, J)
    Jb = O.mean_line_intensity(tb, J)
    for t in range(tb.nline):
        Blu, _ = _einstein_B_lu(p.atom, t)
        assert np.max(np.abs(R_lu[:, t] / (Blu * Jb[:, t]) - 1)) < 1e-13, t


@pytest.mark.parametrize("maker", [S.slab3, S.chromo6])
def test_mean_line_intensity_in_a_planck_field(maker):
    """In the field J = B_nu(T) the profile average is a weighted mean (weights
    w phi >= 0 summing to 1) of B_nu over the line window, so it lies between
    the window's extreme values of B_nu, and close to B_nu0: the window spans
    50 Doppler widths, so |Jbar/B_nu0 - 1| is of order
    50 (1 + h nu0/kT) dnu_D/nu0."""
    p = maker()
    tb = O.setup(p)
    Jb = O.mean_line_intensity(tb, tb.B)
    T = p.atmos.T
    for tr in tb.tr[:tb.nline]:
        Bw = tb.B[:, tr.f0:tr.f1]
        assert np.all(Jb[:, tr.t] >= Bw.min(axis=1) * (1 - 1e-14))
        assert np.all(Jb[:, tr.t] <= Bw.max(axis=1) * (1 + 1e-14))
        _, nu0 = _einstein_B_lu(p.atom, tr.t)
        x = O.HP * nu0 / (O.KB * T)
        dnuD = nu0 / O.CL * np.sqrt(2 * O.KB * T / (p.atom.mass_amu * O.AMU_G))
        bound = 50 * (1 + x) * dnuD / nu0
        assert np.all(np.abs(Jb[:, tr.t] / O.planck(nu0, T) - 1) < bound), tr.t


@pytest.mark.parametrize("maker", [S.slab3, S.chromo6])
def test_detailed_balance_at_planck_field(maker):
    """With I = B_nu(T) everywhere and n = n*, every transition is in detailed
    balance (Eqs. Rij, Rji, gij and the collision rates): bound-free exactly,
    bound-bound to O(h dnu_D / kT); the conservation rows vanish."""
    tb = O.setup(maker())
    r = O.residual(tb, tb.nstar, I_override=tb.B)
    assert np.max(r.rho) < 1e-7
    for t in range(tb.ntr):
        l, u = tb.lo[t], tb.up[t]
        kap = tb.nstar[:, l] * (tb.C_lu[:, t] + r.R_lu[:, t]) - tb.nstar[:, u] * (tb.C_ul[:, t] + r.R_ul[:, t])
        gross = tb.nstar[:, l] * (tb.C_lu[:, t] + r.R_lu[:, t])
        tol = 1e-13 if t >= tb.nline else 1e-8
        assert np.max(np.abs(kap / gross)) < tol, t


# ------------------------------------------------------- derivatives, precond.

@pytest.fixture(scope="module")
def tiny_tb():
    return O.setup(S.tiny())


def _mid_populations(tb):
    rng = np.random.default_rng(11)
    return tb.nstar * np.exp(0.3 * rng.standard_normal(tb.nstar.shape))


def test_jvp_and_preconditioner_against_complex_step(tiny_tb):
    """Brute-force Jacobian by complex step (Eq. complex) on a tiny grid:
    the forward-difference product of Eq. fordif agrees to ~1e-7, and the
    analytic block-Jacobi preconditioner (Sect. 2.5.2 first solution, App. A.2)
    equals the diagonal blocks exactly when there is no background scattering."""
    tb = tiny_tb
    n = _mid_populations(tb)
    r = O.residual(tb, n, want_P=True)
    Jm = O.jacobian_complex_step(tb, n, rows=r.rows)
    N = n.size
    L = tb.nlev
    for k in range(tb.nz):
        blk = Jm[k * L:(k + 1) * L, k * L:(k + 1) * L]
        scale = np.abs(blk).max()
        assert np.max(np.abs(r.P[k] - blk)) < 1e-11 * scale, k
    rng = np.random.default_rng(5)
    v = rng.standard_normal(n.shape) * n
    eps = 1e-7
    Jv = O.jvp_fd(tb, n, v, r.F, eps, rows=r.rows)
    ref = (Jm @ v.ravel()).reshape(n.shape)
    assert np.max(np.abs(Jv - ref)) < 1e-5 * np.max(np.abs(ref))
    # the Jacobian is not block diagonal: radiation couples depths
    off = Jm.copy()
    for k in range(tb.nz):
        off[k * L:(k + 1) * L, k * L:(k + 1) * L] = 0
    assert np.abs(off).max() > 1e-6 * np.abs(Jm).max()
    assert N == tb.nz * L


def test_conservation_rows_in_jacobian(tiny_tb):
    """Conservation rows have derivative -1 on every level of their own depth
    and 0 elsewhere (Sect. 2.5.1)."""
    tb = tiny_tb
    n = _mid_populations(tb)
    r = O.residual(tb, n)
    Jm = O.jacobian_complex_step(tb, n, rows=r.rows)
    L = tb.nlev
    for k in range(tb.nz):
        row = Jm[k * L + r.rows[k]]
        expect = np.zeros(Jm.shape[1])
        expect[k * L:(k + 1) * L] = -1.0
        assert np.array_equal(row, expect)


def _richardson_product(tb, n, v, rows, h):
    """Central differences of the real residual at steps h and h/2, combined
    so that the O(h^2) error cancels (error O(h^4))."""
    def central(s):
        Fp = O.residual(tb, n + s * v, rows=rows).F
        Fm = O.residual(tb, n - s * v, rows=rows).F
        return (Fp - Fm) / (2 * s)
    return (4 * central(h / 2) - central(h)) / 3


@pytest.mark.parametrize("maker", ["tiny", "slab3"])
def test_complex_step_product_matches_extrapolated_differences(maker, tiny_tb):
    """Complex-step product of Eq. complex (step 1e-200, Sect. 2.4.2) against
    Richardson-extrapolated central differences of the real residual, which
    share none of its complex arithmetic: a dropped or mis-signed term in
    the derivative of any step of Algorithm 1 (opacity, formal solution,
    rates, assembly) shows up far above the 1e-10 the differences reach."""
    tb = tiny_tb if maker == "tiny" else O.setup(S.slab3())
    n = _mid_populations(tb)
    rows = O.conservation_rows(n)
    rng = np.random.default_rng(7)
    v = rng.standard_normal(n.shape) * n
    cs = O.jvp_complex_step(tb, n, v, rows=rows)
    ref = _richardson_product(tb, n, v, rows, 2e-3)
    scale = np.abs(ref).max()
    assert np.max(np.abs(cs - ref)) < 1e-10 * scale
    # the coupling through the radiation field is in it: with J held fixed
    # the product differs by far more than that tolerance
    r = O.residual(tb, n)
    Ff = O.residual(tb, n + 1j * 1e-200 * v, rows=rows, I_override=r.J).F.imag / 1e-200
    assert np.max(np.abs(Ff - cs)) > 1e-4 * scale


def test_complex_step_with_frozen_radiation_is_rate_matrix(tiny_tb):
    """With J held fixed, F is linear in n (Eqs. residuals_1/2): the complex
    step returns the rate matrix times v, and -sum v on the conservation rows
    (Sect. 2.5.1)."""
    tb = tiny_tb
    n = _mid_populations(tb)
    r = O.residual(tb, n)
    rng = np.random.default_rng(8)
    v = rng.standard_normal(n.shape) * n
    Ff = O.residual(tb, n + 1j * 1e-200 * v, rows=r.rows, I_override=r.J).F.imag / 1e-200
    L = tb.nlev
    for k in range(tb.nz):
        A = np.zeros((L, L))  # A[i, j]: rate from level j into level i, minus outflow on the diagonal
        for t in range(tb.ntr):
            lo, up = tb.lo[t], tb.up[t]
            ul = tb.C_lu[k, t] + r.R_lu[k, t]
            dl = tb.C_ul[k, t] + r.R_ul[k, t]
            A[lo, lo] += ul
            A[up, lo] -= ul
            A[lo, up] -= dl
            A[up, up] += dl
        expect = A @ v[k]
        expect[r.rows[k]] = -v[k].sum()
        assert np.allclose(Ff[k], expect, rtol=1e-12, atol=1e-12 * np.abs(expect).max()), k


def test_complex_step_product_is_linear(tiny_tb):
    """The complex-step product is exact to rounding, so it is linear in v
    (a forward difference is not: its error depends on the step and on v)."""
    tb = tiny_tb
    n = _mid_populations(tb)
    rows = O.conservation_rows(n)
    rng = np.random.default_rng(9)
    a = rng.standard_normal(n.shape) * n
    b = rng.standard_normal(n.shape) * n
    lhs = O.jvp_complex_step(tb, n, 2.0 * a - 3.0 * b, rows=rows)
    rhs = 2.0 * O.jvp_complex_step(tb, n, a, rows=rows) - 3.0 * O.jvp_complex_step(tb, n, b, rows=rows)
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.abs(rhs).max()


def test_gmres_solves_small_system():
    rng = np.random.default_rng(2)
    A = np.eye(40) + 0.3 * rng.standard_normal((40, 40)) / np.sqrt(40)
    b = rng.standard_normal(40)
    x, it, rel = O.gmres(lambda v: A @ v, b, rtol=1e-12, m=10, maxit=400)
    assert rel <= 1e-12
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-11)


def test_bicgstab_solves_small_system():
    """The oracle's BiCGSTAB against a direct solve of a nonsymmetric
    system (a library routine, not the method under test)."""
    rng = np.random.default_rng(3)
    A = np.eye(40) + 0.3 * rng.standard_normal((40, 40)) / np.sqrt(40)
    b = rng.standard_normal(40)
    x, k, rel = O.bicgstab(lambda v: A @ v, b, rtol=1e-12, maxit=400)
    assert rel <= 1e-12
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("method", ["gmres", "bicgstab"])
def test_krylov_from_a_nonzero_initial_guess(method):
    """Both inner solvers started from a nonzero x0 (Algorithm 2's second
    initial guess) against a direct solve; the start costs one product (GMRES
    does not count the products of its restarts), and from the exact
    solution the first iteration already meets the tolerance."""
    rng = np.random.default_rng(6)
    A = np.eye(40) + 0.3 * rng.standard_normal((40, 40)) / np.sqrt(40)
    b = rng.standard_normal(40)
    xs = np.linalg.solve(A, b)
    x0 = xs + 0.1 * rng.standard_normal(40)
    calls = []

    def mv(v):
        calls.append(1)
        return A @ v
    if method == "gmres":
        x, k, rel = O.gmres(mv, b, rtol=1e-12, m=10, maxit=400, x0=x0)
    else:
        x, k, rel = O.bicgstab(mv, b, rtol=1e-12, maxit=400, x0=x0)
    assert k <= len(calls) and rel <= 1e-12
    if method == "bicgstab":
        assert k == len(calls)
    assert np.allclose(x, xs, rtol=1e-9, atol=1e-11)
    fn = O.gmres if method == "gmres" else O.bicgstab
    x, k, rel = fn(lambda v: A @ v, b, rtol=1e-10, maxit=10, x0=xs)
    assert k <= 2 and rel <= 1e-10 and np.allclose(x, xs, rtol=1e-12)


def test_bicgstab_two_eigenvalues_one_iteration():
    """A diagonal operator with two distinct eigenvalues: the first
    iteration's step (BiCG direction plus the minimal-residual omega) already
    spans its minimal polynomial, so the residual vanishes after two
    products, to rounding."""
    d = np.where(np.arange(30) % 2 == 0, 2.0, 5.0)
    b = np.linspace(1.0, 2.0, 30)
    x, k, rel = O.bicgstab(lambda v: d * v, b, rtol=1e-13, maxit=50)
    assert k <= 4 and rel <= 1e-13
    assert np.allclose(x, b / d, rtol=1e-12)


def test_zero_radiation_guess_satisfies_rate_equations():
    """The radiation-free guess solves F = 0 with J forced to zero."""
    tb = O.setup(S.chromo6(nz=20, nnu=120))
    n0 = O.zero_radiation_guess(tb)
    r = O.residual(tb, n0, I_override=np.zeros((tb.nz, tb.nnu)))
    assert np.max(r.rho) < 1e-12
    assert np.all(n0 > 0)


# ------------------------------------------------------------------- solves

def test_jfnk_root_equals_dense_newton_root(tiny_tb):
    """Dense Newton with the brute-force Jacobian and JFNK reach the same root
    (Sect. 3.2: both solve the same F = 0)."""
    tb = tiny_tb
    s = O.solve(tb, ftol=1e-13, rtol=1e-8, maxiter=40)
    assert s.converged
    nd, _ = O.dense_newton(tb, tb.nstar, ftol=1e-13)
    assert np.max(np.abs(s.n / nd - 1)) < 1e-11
    # particle conservation at convergence
    assert np.max(np.abs(s.n.sum(axis=1) / tb.ntot - 1)) < 1e-13


def test_jfnk_bicgstab_root_equals_gmres_root(tiny_tb):
    """Both inner solvers of the paper (Sect. 3.2: they converge to the same
    solution) reach the dense-Newton root."""
    tb = tiny_tb
    s = O.solve(tb, ftol=1e-13, rtol=1e-8, maxiter=40, krylov="bicgstab")
    assert s.converged
    nd, _ = O.dense_newton(tb, tb.nstar, ftol=1e-13)
    assert np.max(np.abs(s.n / nd - 1)) < 1e-11


def test_jfnk_preconditioned_initial_guess_root(tiny_tb):
    """JFNK whose Krylov solves start from x0 = -P^-1 F (Algorithm 2) reaches
    the dense-Newton root with both inner solvers."""
    tb = tiny_tb
    nd, _ = O.dense_newton(tb, tb.nstar, ftol=1e-13)
    for kr in ("gmres", "bicgstab"):
        s = O.solve(tb, ftol=1e-13, rtol=1e-8, maxiter=40, krylov=kr, krylov_x0="precond")
        assert s.converged, kr
        assert np.max(np.abs(s.n / nd - 1)) < 1e-11, kr


def test_jfnk_complex_step_root_equals_dense_newton_root(tiny_tb):
    """JFNK with complex-step products (Eq. complex, the products the paper's
    runs use) reaches the dense-Newton root, with both inner solvers."""
    tb = tiny_tb
    nd, _ = O.dense_newton(tb, tb.nstar, ftol=1e-13)
    for kr in ("gmres", "bicgstab"):
        s = O.solve(tb, ftol=1e-13, rtol=1e-8, maxiter=40, krylov=kr, jv="complex")
        assert s.converged, kr
        assert np.max(np.abs(s.n / nd - 1)) < 1e-11, kr


def test_collisional_limit_gives_lte():
    """Collision-dominated rates drive the solution to Saha-Boltzmann LTE."""
    p = S.slab3()
    p.C_up = p.C_up * 1e11
    tb = O.setup(p)
    n0 = tb.nstar * np.exp(0.2 * np.random.default_rng(0).standard_normal(tb.nstar.shape))
    s = O.solve(tb, n0=n0, ftol=1e-12, rtol=1e-6)
    assert s.converged
    assert np.max(np.abs(s.n / tb.nstar - 1)) < 1e-6


def _surface_ratio(eps, ppd):
    p = S.two_level(eps, pts_per_decade=ppd)
    tb = O.setup(p)
    s = O.solve(tb, ftol=1e-10, rtol=1e-6, maxiter=60)
    assert s.converged
    n, a = s.n, p.atom
    nu0 = (a.E[1] - a.E[0]) / O.HP
    Sl = 2 * O.HP * nu0 ** 3 / O.CL ** 2 / (n[:, 0] * a.g[1] / (n[:, 1] * a.g[0]) - 1)
    return Sl[0] / O.planck(nu0, p.atmos.T[0]) / math.sqrt(eps)


@pytest.mark.slow
@pytest.mark.parametrize("eps,tol", [(1e-2, 0.02), (1e-3, 0.05), (1e-4, 0.12)])
def test_sqrt_eps_law(eps, tol):
    """Two-level atom, isothermal, no continuum: the surface line source
    function tends to sqrt(eps) B (the classic scattering-dominated limit the
    NLTE solution must reproduce); the discretisation error shrinks when the
    depth grid is refined from 10 to 20 points per decade."""
    coarse = _surface_ratio(eps, 10)
    fine = _surface_ratio(eps, 20)
    assert abs(fine - 1) < tol, (coarse, fine)
    assert abs(fine - 1) < 0.6 * abs(coarse - 1), (coarse, fine)


@pytest.mark.slow
def test_scattering_forward_difference_root_equals_complex_step_root():
    """Background (Thomson) scattering makes F depend on the lagged J-dagger
    (Sect. 2.1.1).  JFNK with forward-difference products (Eq. fordif) and
    with complex-step products (Eq. complex) reaches the same root only if
    F(n), the products and the line search of a Newton step share one
    J-dagger; at the root J-dagger is self-consistent (J(n; J-dagger) =
    J-dagger)."""
    tb = O.setup(S.chromo6(nz=40, nnu=200, thomson=True))
    assert np.any(tb.chi_sca > 0)
    fd = O.solve(tb, ftol=1e-12, rtol=1e-4, maxiter=40, jv="fd")
    cs = O.solve(tb, ftol=1e-12, rtol=1e-4, maxiter=40, jv="complex")
    assert fd.converged and cs.converged
    assert np.max(np.abs(fd.n / cs.n - 1)) < 1e-10
    r = O.residual(tb, cs.n, Jdag=cs.J)
    assert np.max(r.rho) <= 1e-12
    assert np.max(np.abs(r.J / cs.J - 1)) < 1e-9


def test_per_depth_correction_limit():
    """Sect. 2.2.2 limits the Newton correction depth by depth: with the
    factor-3 reading, every level of n + lambda_k dn stays within
    [n/3, 3n] and stays positive, lambda_k is 1 when the full step already
    does, and otherwise the bound is reached by one level of that depth."""
    rng = np.random.default_rng(21)
    n = 10.0 ** rng.uniform(-3, 12, (200, 6))
    dn = n * rng.normal(0.0, 1.5, n.shape)
    lam = O.positivity_limit(n, dn)
    assert lam.shape == (200,) and np.all((lam > 0) & (lam <= 1))
    new = n + lam[:, None] * dn
    r = new / n
    assert np.all(r >= 1 / 3 - 1e-12) and np.all(r <= 3 + 1e-12) and np.all(new > 0)
    full = n + dn
    ok = np.all((full / n >= 1 / 3) & (full / n <= 3), axis=1)
    assert np.all(lam[ok] == 1.0)
    tight = np.min(np.minimum(np.abs(r - 1 / 3), np.abs(r - 3)), axis=1)
    assert np.all(tight[~ok] < 1e-12) and np.any(~ok)
