"""Pins of the oracle's velocity-field path (Sect. 3.5: line profiles
Doppler-shifted by the velocity component along each ray, so opacity, formal
solution and line rates are taken ray by ray).

Each check is fixed by something other than the code under test: the static
path (zero velocity), Galilean invariance (a uniform flow shifts each ray's
spectrum by nu0 s mu v / c and leaves the populations unchanged up to the
discretisation), profile normalisation, the Einstein relations, detailed
balance and the brute-force complex-step Jacobian."""
import copy

import numpy as np
import pytest

from oracle import nlte_oracle as O
from paper_2406_17234_amd import synth as S


def _with_velocity(p, v):
    q = copy.deepcopy(p)
    q.atmos.vlos = np.broadcast_to(np.asarray(v, dtype=float), (q.atmos.nz,)).copy()
    return q


def _photosphere(v_kms=3.0, nz=60):
    """A 3-level atom in the photospheric part of the chromosphere model
    (temperature falling outwards, so the line is in absorption), uniform
    upward flow of v_kms, frequency grid resolving the shifted cores."""
    atom = S.make_atom(3, 1, 1, name="atom3")
    atm = S.chromosphere(nz=nz, abund=S.ABUND[3], h_top_km=450.0, h_bot_km=-100.0)
    atm.vlos = np.full(atm.nz, v_kms * 1e5)
    grid = S.make_grid(atom, atm, 61, 10, 3, v_max=v_kms * 1e5)
    return S.Problem("photosphere", atom, atm, grid, S.make_collisions(atom, atm), 1)


def _mid(tb, seed=11):
    rng = np.random.default_rng(seed)
    return tb.nstar * np.exp(0.3 * rng.standard_normal(tb.nstar.shape))


@pytest.mark.parametrize("maker", [S.tiny, lambda: S.chromo6(nz=24, nnu=200, nmu=3)])
def test_zero_velocity_is_the_static_problem(maker):
    """A velocity field of zeros runs the ray-by-ray path and returns the
    static F, J, rates, Jbar and preconditioner to rounding."""
    p = maker()
    tb = O.setup(p)
    tv = O.setup(_with_velocity(p, 0.0))
    assert tv.vel and not tb.vel
    n = _mid(tb)
    a = O.residual(tb, n, want_P=True)
    b = O.residual(tv, n, want_P=True)
    assert np.max(np.abs(a.F - b.F) / a.G) < 1e-14
    for name in ("J", "R_lu", "R_ul", "Jbar", "P"):
        x, y = getattr(a, name), getattr(b, name)
        assert np.max(np.abs(x - y)) <= 1e-14 * np.max(np.abs(x)), name


def test_uniform_flow_shifts_each_ray():
    """Galilean invariance at fixed populations: with a uniform upward flow v
    each ray's intensity is the static one shifted in frequency by
    nu0 s mu v / c, s = +1 for outgoing and -1 for ingoing rays (to the
    interpolation error of the grid, a few per cent of the line depth); the
    opposite shift, or none, is far off."""
    v = 3e5
    p = _photosphere(v / 1e5)
    q = copy.deepcopy(p)
    q.atmos.vlos = np.zeros(p.atmos.nz)
    tb, t0 = O.setup(p), O.setup(q)
    r, r0 = O.residual(tb, tb.nstar), O.residual(t0, t0.nstar)
    tr = tb.tr[0]
    nu = tb.nu[tr.f0:tr.f1]
    for ray in range(tb.nray):
        s = 1.0 if ray < tb.nmu else -1.0
        shift = tr.nu0 * s * tb.mu[ray % tb.nmu] * v / O.CL
        for k in ([0] if s > 0 else [5, 30]):  # emergent, and two depths for ingoing rays
            I = r.I[ray, k, tr.f0:tr.f1]
            I0 = r0.I[ray, k, tr.f0:tr.f1]
            depth = I0.max() - I0.min()
            assert depth > 0.4 * I0.max()
            good = np.max(np.abs(I - np.interp(nu - shift, nu, I0))) / depth
            wrong = np.max(np.abs(I - np.interp(nu + shift, nu, I0))) / depth
            still = np.max(np.abs(I - I0)) / depth
            assert good < 0.04, (ray, k, good)
            assert wrong > 0.3 and still > 0.2, (ray, k, wrong, still)


def test_uniform_flow_leaves_the_populations():
    """The root with a uniform flow equals the static root up to the
    discretisation of the shifted profiles (below 1 per cent here), while a
    velocity gradient of the same amplitude changes it by tens of per cent."""
    p = _photosphere(3.0)
    q = copy.deepcopy(p)
    q.atmos.vlos = np.zeros(p.atmos.nz)
    g = copy.deepcopy(p)
    g.atmos.vlos = S.velocity_step(-p.atmos.z / 1e5, 3.0, 200.0, 50.0)
    roots = []
    for prob in (p, q, g):
        s = O.solve(O.setup(prob), ftol=1e-10, rtol=1e-6, maxiter=50)
        assert s.converged
        roots.append(s.n)
    assert np.max(np.abs(roots[0] / roots[1] - 1)) < 1e-2
    assert np.max(np.abs(roots[2] / roots[1] - 1)) > 0.1


def test_flat_field_and_einstein_relation_with_flow():
    """Every ray's profile is normalised on the window, and the ray weights
    sum to one: an isotropic field constant in frequency gives Jbar = J at
    every depth; R_lu = B_lu Jbar holds for any field (Eq. Rij with V of
    Eq. Vij), with B_lu from the Einstein relations."""
    p = S.chromo6_vel(nz=40, nnu=300, nmu=3)
    tb = O.setup(p)
    assert tb.vel
    c = np.geomspace(1e-3, 1e3, tb.nz)[:, None]
    r = O.residual(tb, tb.nstar, I_override=c * np.ones((1, tb.nnu)))
    assert np.max(np.abs(r.Jbar / c - 1)) < 1e-14
    rng = np.random.default_rng(4)
    r = O.residual(tb, tb.nstar, I_override=tb.B * np.exp(rng.standard_normal(tb.B.shape)))
    for t in range(tb.nline):
        lo, up = p.atom.line_lo[t], p.atom.line_up[t]
        nu0 = (p.atom.E[up] - p.atom.E[lo]) / O.HP
        Blu = p.atom.g[up] / p.atom.g[lo] * p.atom.A_ul[t] * O.CL ** 2 / (2 * O.HP * nu0 ** 3)
        assert np.max(np.abs(r.R_lu[:, t] / (Blu * r.Jbar[:, t]) - 1)) < 1e-13, t


def test_detailed_balance_with_flow():
    """I = B_nu(T) on every ray and n = n*: detailed balance holds ray by
    ray, bound-free exactly and bound-bound to O(h dnu_D / kT), so the flow
    does not move LTE."""
    tb = O.setup(S.chromo6_vel(nz=40, nnu=300, nmu=3))
    r = O.residual(tb, tb.nstar, I_override=tb.B)
    assert np.max(r.rho) < 1e-7
    for t in range(tb.ntr):
        l, u = tb.lo[t], tb.up[t]
        kap = tb.nstar[:, l] * (tb.C_lu[:, t] + r.R_lu[:, t]) - tb.nstar[:, u] * (tb.C_ul[:, t] + r.R_ul[:, t])
        gross = tb.nstar[:, l] * (tb.C_lu[:, t] + r.R_lu[:, t])
        assert np.max(np.abs(kap / gross)) < (1e-13 if t >= tb.nline else 1e-7), t


def _tiny_flow():
    p = S.tiny()
    return _with_velocity(p, np.linspace(3e5, -2e5, p.atmos.nz))


def test_preconditioner_with_flow_is_the_jacobian_diagonal():
    """With a velocity gradient the preconditioner blocks (Sect. 2.5.2 first
    solution, App. A.2, each ray with its own opacity and profile) equal the
    diagonal blocks of the brute-force complex-step Jacobian."""
    tb = O.setup(_tiny_flow())
    n = _mid(tb)
    r = O.residual(tb, n, want_P=True)
    Jm = O.jacobian_complex_step(tb, n, rows=r.rows)
    L = tb.nlev
    for k in range(tb.nz):
        blk = Jm[k * L:(k + 1) * L, k * L:(k + 1) * L]
        assert np.max(np.abs(r.P[k] - blk)) < 1e-11 * np.abs(blk).max(), k
    # the flow matters: the static problem has other blocks
    p0 = copy.deepcopy(_tiny_flow())
    p0.atmos.vlos = None
    P0 = O.residual(O.setup(p0), n, want_P=True).P
    assert np.max(np.abs(P0 - r.P)) > 1e-6 * np.abs(r.P).max()


def test_complex_step_with_flow_matches_extrapolated_differences():
    """Complex-step product (Eq. complex) through the ray-by-ray path against
    Richardson-extrapolated central differences of the real residual."""
    tb = O.setup(_tiny_flow())
    n = _mid(tb)
    rows = O.conservation_rows(n)
    rng = np.random.default_rng(8)
    v = rng.standard_normal(n.shape) * n
    cs = O.jvp_complex_step(tb, n, v, rows=rows)
    h = 1e-3

    def central(step):
        return (O.residual(tb, n + step * v, rows=rows).F - O.residual(tb, n - step * v, rows=rows).F) / (2 * step)

    rich = (4.0 * central(h / 2) - central(h)) / 3.0
    assert np.max(np.abs(cs - rich)) < 1e-6 * np.max(np.abs(cs))


def test_flow_root_by_jfnk_equals_dense_newton():
    """JFNK with forward-difference products reaches the root that Newton
    with the dense complex-step Jacobian reaches, with a velocity gradient."""
    tb = O.setup(_tiny_flow())
    s = O.solve(tb, ftol=1e-13, rtol=1e-8, maxiter=40)
    assert s.converged
    n = tb.nstar.copy()
    for _ in range(30):
        r = O.residual(tb, n)
        if np.max(r.rho) < 1e-13:
            break
        Jm = O.jacobian_complex_step(tb, n, rows=r.rows)
        n = n + np.linalg.solve(Jm, -r.F.ravel()).reshape(n.shape)
    assert np.max(np.abs(n / s.n - 1)) < 1e-10
