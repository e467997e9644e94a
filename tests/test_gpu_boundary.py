"""Boundary inputs of the C ABI on the device against the FP64 oracle:
caller background emissivity and frequency weights, background (Thomson)
scattering with its lagged J-dagger, a solve resumed from (n, J), the
preconditioned Krylov initial guess of Algorithm 2, and non-finite or
non-positive populations."""
import copy

import numpy as np
import pytest

from oracle import nlte_oracle as O
from paper_2406_17234_amd import synth as S
from tests.helpers import maxrel, perturbed, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_2406_17234_amd import nlte
    return nlte.Context(0)


def _custom_inputs():
    """chromo6 with a caller background emissivity (a hotter Planck function
    times a smooth factor, zero at two depths) and caller frequency weights
    (trapezoid-like with a smooth modulation)."""
    p = S.chromo6(nz=40, nnu=240)
    nu = p.grid.nu
    T = p.atmos.T
    fac = 1.0 + 0.5 * np.sin(np.linspace(0.0, 7.0, len(nu)))[None, :]
    eta = p.atmos.chi_c[:, None] * O.planck(nu[None, :], 1.08 * T[:, None]) * fac
    eta[3] = 0.0
    eta[17] = 0.0
    p.atmos.eta_c = eta
    g = np.gradient(nu)
    p.grid.w_nu = g * (1.0 + 0.2 * np.cos(np.linspace(0.0, 11.0, len(nu))))
    return p


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_residual_with_caller_emissivity_and_weights(ctx, precision):
    from paper_2406_17234_amd import nlte
    p = _custom_inputs()
    tb = O.setup(p)
    n = perturbed(tb.nstar, seed=3, scale=0.3)
    ref = O.residual(tb, n)
    prec = nlte.FP64 if precision == "fp64" else nlte.FP32_FORM
    print(f"[case] residual eta_c/w_nu {precision} dims={p.dims}", flush=True)
    col = nlte.Column(ctx, p, precision=prec)
    out = col.residual(to_dev(n), want_J=True, want_R=True, want_Jbar=True)
    tolF, tolJ = (1e-12, 1e-12) if precision == "fp64" else (1e-4, 1e-4)
    assert np.max(np.abs(to_np(out["F"]) - ref.F) / ref.G) < tolF
    assert maxrel(to_np(out["J"]), ref.J, floor=1e-30 * np.abs(ref.J).max()) < tolJ
    R = to_np(out["R"])
    assert maxrel(R[:, :, 0], ref.R_lu) < tolJ
    assert maxrel(R[:, :, 1], ref.R_ul) < tolJ
    assert maxrel(to_np(out["Jbar"]), ref.Jbar) < tolJ
    # the inputs matter: the default emissivity and weights give another F
    d = copy.deepcopy(p)
    d.atmos.eta_c = None
    d.grid.w_nu = None
    other = O.residual(O.setup(d), n)
    assert np.max(np.abs(other.F - ref.F) / ref.G) > 1e-6


_SCA = {}


def _sca_root():
    if "root" not in _SCA:
        p = S.chromo6(nz=40, nnu=200, thomson=True)
        tb = O.setup(p)
        s = O.solve(tb, ftol=1e-12, rtol=1e-6, maxiter=60)
        assert s.converged
        _SCA["root"] = (p, tb, s)
    return _SCA["root"]


@pytest.mark.parametrize("jv", ["fd", "tangent"])
def test_scattering_solve_matches_oracle_root(ctx, jv):
    """Background Thomson scattering: the device solve (one J-dagger per
    Newton step) reaches the oracle root and a self-consistent J-dagger."""
    from paper_2406_17234_amd import nlte
    p, tb, ref = _sca_root()
    print(f"[case] thomson solve jv={jv} dims={p.dims}", flush=True)
    col = nlte.Column(ctx, p)
    jvm = nlte.JV_FD if jv == "fd" else nlte.JV_TANGENT
    n, J, st, rc = col.solve(ftol=1e-12, rtol=1e-6, maxiter=60, want_J=True, jv_method=jvm)
    print(st, flush=True)
    assert rc == 0 and st["status"] == 0
    assert maxrel(to_np(n), ref.n) < 1e-10
    assert maxrel(to_np(J), ref.J) < 1e-9


def test_solve_resumes_from_n_and_J(ctx):
    """Algorithm 2 takes n0 and an initial estimate of J: a solve stopped
    after 3 Newton iterations and restarted from its (n, J) ends on the same
    populations, bit for bit, as the uninterrupted solve (background
    scattering, so J-dagger matters)."""
    from paper_2406_17234_amd import nlte
    p, tb, ref = _sca_root()
    col = nlte.Column(ctx, p)
    full, _, st_full, rc = col.solve(ftol=1e-12, rtol=1e-4, maxiter=60)
    assert rc == 0
    assert st_full["newton_iters"] > 3
    part, Jp, st_p, rc_p = col.solve(ftol=1e-12, rtol=1e-4, maxiter=3, want_J=True)
    assert rc_p == nlte.NLTE_E_NOCONV and st_p["newton_iters"] == 3
    res, _, st_r, rc_r = col.solve(n0=part, J0=Jp, init=0, ftol=1e-12, rtol=1e-4, maxiter=60)
    assert rc_r == 0
    assert st_r["newton_iters"] + 3 == st_full["newton_iters"]
    assert np.array_equal(to_np(res), to_np(full))
    # without J0 the restart uses B_nu(T) and takes another path to the root
    res2, _, st2, rc2 = col.solve(n0=part, init=0, ftol=1e-12, rtol=1e-4, maxiter=60)
    assert rc2 == 0 and maxrel(to_np(res2), ref.n) < 1e-10
    assert not np.array_equal(to_np(res2), to_np(full))


@pytest.mark.parametrize("method", ["gmres", "bicgstab"])
def test_preconditioned_initial_guess(ctx, method):
    """Krylov solves started from x0 = -P^-1 F (Algorithm 2) reach the oracle
    root; the oracle with the same option reaches it too."""
    from paper_2406_17234_amd import nlte
    p = S.chromo6(nz=40, nnu=300)
    tb = O.setup(p)
    kr = "gmres" if method == "gmres" else "bicgstab"
    # both sides one quadratic step past 1e-12 (a stop just under 1e-12 can
    # leave ~1e-10 of the last correction in the populations)
    ref = O.solve(tb, ftol=1e-14, rtol=1e-6, maxiter=60, krylov=kr, krylov_x0="precond")
    assert ref.converged
    col = nlte.Column(ctx, p)
    km = nlte.KRYLOV_GMRES if method == "gmres" else nlte.KRYLOV_BICGSTAB
    print(f"[case] x0=precond {method}", flush=True)
    n, _, st, rc = col.solve(ftol=1e-14, rtol=1e-6, maxiter=60, krylov_method=km, krylov_x0=1)
    print(st, flush=True)
    assert rc == 0 and st["status"] == 0
    assert maxrel(to_np(n), ref.n) < 1e-10
    # one extra product per Newton iteration is counted
    n0, _, st0, _ = col.solve(ftol=1e-14, rtol=1e-6, maxiter=60, krylov_method=km)
    assert maxrel(to_np(n0), ref.n) < 1e-10


def test_nonfinite_populations_rejected(ctx):
    from paper_2406_17234_amd import nlte
    p = S.slab3()
    tb = O.setup(p)
    col = nlte.Column(ctx, p)
    for bad in (np.nan, np.inf, -1.0, 0.0):
        n = tb.nstar.copy()
        n[5, 1] = bad
        with pytest.raises(nlte.NLTEError) as e:
            col.residual(to_dev(n))
        assert e.value.status == nlte.NLTE_E_NONFINITE
        with pytest.raises(nlte.NLTEError) as e:
            col.jvp(to_dev(n), to_dev(np.ones_like(n)), 1e-6)
        assert e.value.status == nlte.NLTE_E_NONFINITE
    # a solve started from NaN populations stops with NONFINITE, not a hang
    n = tb.nstar.copy()
    n[7, 0] = np.nan
    out, _, st, rc = col.solve(n0=to_dev(n), init=0, maxiter=5)
    assert rc == nlte.NLTE_E_NOCONV and st["status"] == nlte.NLTE_E_NONFINITE
    # the column still works afterwards
    good = col.residual(to_dev(tb.nstar))
    assert np.all(np.isfinite(to_np(good["F"])))
