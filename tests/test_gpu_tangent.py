"""Tangent-linear Jacobian-vector products (Sect. 2.4.2, Eq. complex) on the
device, against the oracle's complex-step product Im F(n + i h v)/h with
h = 1e-200, and JFNK solves that use them."""
import numpy as np
import pytest

from oracle import nlte_oracle as O
from paper_2406_17234_amd import synth as S
from tests.helpers import maxrel, perturbed, require_gpu, to_dev, to_np
from tests.test_gpu_solve import CASES, oracle_root

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_2406_17234_amd import nlte
    return nlte.Context(0)


def _case(name, seed):
    prob = CASES[name]()
    tb = O.setup(prob)
    n = perturbed(tb.nstar, seed=seed, scale=0.2)
    rng = np.random.default_rng(seed + 100)
    v = rng.standard_normal(n.shape) * n
    return prob, tb, n, v


# The product is the exact derivative on both sides; only rounding differs
# (sums in another order, the series of the segment coefficients evaluated
# differently), so FP64 columns agree to 1e-13 of the largest component.
# FP32-form columns compute the tangent in FP64 but take the rates of n from
# their own FP32-form evaluation (J to ~1e-6 relative).
@pytest.mark.parametrize("name,flags,tol", [
    ("tiny", "fp64", 1e-13),
    ("slab3", "fp64", 1e-13),
    ("chromo6_small", "fp64", 1e-13),
    ("chromo6_small", "scan", 1e-13),
    ("chromo6", "fp64", 1e-13),
    ("chromo6_small", "fp32", 1e-6),
])
def test_tangent_product_matches_oracle_complex_step(ctx, name, flags, tol):
    from paper_2406_17234_amd import nlte
    prec = {"fp64": nlte.FP64, "scan": nlte.FP64 | nlte.DEPTH_SCAN, "fp32": nlte.FP32_FORM}[flags]
    prob, tb, n, v = _case(name, 71)
    print(f"[case] tangent product {name} {flags} dims={prob.dims}", flush=True)
    ref = O.jvp_complex_step(tb, n, v)
    col = nlte.Column(ctx, prob, precision=prec)
    Jv = to_np(col.jvp_tangent(to_dev(n), to_dev(v)))
    err = np.max(np.abs(Jv - ref)) / np.max(np.abs(ref))
    print(f"  max err / max |Jv| = {err:.3e}", flush=True)
    assert err < tol
    # the rows: -sum v on each conservation row, exactly as the oracle's
    rows = O.conservation_rows(n)
    k = np.arange(tb.nz)
    assert np.allclose(Jv[k, rows], -v.sum(axis=1), rtol=1e-14, atol=0)
    col.close()


def _sixteen():
    from tests.test_gpu_edges import _sixteen_levels
    return _sixteen_levels()


@pytest.mark.parametrize("name,maker", [
    ("smallest column, one angle", lambda: S.tiny(nz=3, nmu=1, nline_pts=3, nbf_pts=2)),
    ("eight angles", lambda: S.tiny(nmu=8)),
    ("16 levels, 24 lines, 15 edges", _sixteen),
])
def test_tangent_product_at_the_size_limits(ctx, name, maker):
    """The angle counts at both ends of the range (each its own kernel
    instantiation), the smallest column and the largest atom."""
    from paper_2406_17234_amd import nlte
    prob = maker()
    tb = O.setup(prob)
    n = perturbed(tb.nstar, seed=73, scale=0.2)
    v = np.random.default_rng(173).standard_normal(n.shape) * n
    print(f"[case] tangent product {name} dims={prob.dims}", flush=True)
    ref = O.jvp_complex_step(tb, n, v)
    col = nlte.Column(ctx, prob, precision=nlte.FP64)
    Jv = to_np(col.jvp_tangent(to_dev(n), to_dev(v)))
    err = np.max(np.abs(Jv - ref)) / np.max(np.abs(ref))
    print(f"  max err / max |Jv| = {err:.3e}", flush=True)
    assert err < 1e-13
    col.close()


def test_tangent_product_is_linear_and_close_to_forward_difference(ctx):
    """Exact to rounding, so linear in v; the forward difference of Eq. fordif
    approaches it to its truncation error."""
    from paper_2406_17234_amd import nlte
    prob, tb, n, v = _case("chromo6_small", 72)
    w = np.random.default_rng(5).standard_normal(n.shape) * n
    col = nlte.Column(ctx, prob)
    nd = to_dev(n)
    a = to_np(col.jvp_tangent(nd, to_dev(v)))
    b = to_np(col.jvp_tangent(nd, to_dev(w)))
    c = to_np(col.jvp_tangent(nd, to_dev(2.0 * v - 3.0 * w)))
    assert np.max(np.abs(c - (2 * a - 3 * b))) < 1e-12 * np.max(np.abs(c))
    fd = to_np(col.jvp(nd, to_dev(v), 1e-7))
    assert np.max(np.abs(fd - a)) < 1e-5 * np.max(np.abs(a))
    # the column still evaluates residuals as before
    F = to_np(col.residual(nd)["F"])
    r = O.residual(tb, n)
    assert np.max(np.abs(F - r.F) / r.G) < 1e-11
    col.close()


@pytest.mark.parametrize("krylov", [0, 1], ids=["gmres", "bicgstab"])
@pytest.mark.parametrize("name", ["slab3", "chromo6_small"])
def test_tangent_solve_fp64_matches_oracle_root(ctx, name, krylov):
    """JFNK with tangent products (the paper's complex-step scheme) reaches
    the oracle's root with both inner solvers."""
    from paper_2406_17234_amd import nlte
    prob, tb, ref = oracle_root(name, CASES[name])
    print(f"[case] tangent solve {name} krylov={krylov}", flush=True)
    col = nlte.Column(ctx, prob)
    n, _, st, rc = col.solve(ftol=1e-12, rtol=1e-6, maxiter=60, krylov_method=krylov,
                             jv_method=nlte.JV_TANGENT)
    print(st, flush=True)
    assert rc == 0 and st["rho_inf"] <= 1e-12
    assert maxrel(to_np(n), ref.n) < 1e-10
    col.close()


def test_tangent_solve_fp32_form_batch(ctx):
    """Batched FP32-form columns with tangent products (FP64 derivative of
    the FP32-form residual's arithmetic) converge to within 1e-4 of the FP64
    root."""
    from paper_2406_17234_amd import nlte
    prob, tb, ref = oracle_root("chromo6", CASES["chromo6"])
    cols = [nlte.Column(ctx, prob, precision=nlte.FP32_FORM) for _ in range(3)]
    outs, stats, rc = nlte.solve_batch(ctx, cols, ftol=1e-6, rtol=1e-3, maxiter=60,
                                       jv_method=nlte.JV_TANGENT, fp64_fallback=30)
    print(stats[0], flush=True)
    assert rc == 0
    for o, s in zip(outs, stats):
        assert s["status"] == 0
        assert maxrel(to_np(o), ref.n) < 1e-4


def test_unknown_jv_method_rejected(ctx):
    from paper_2406_17234_amd import nlte
    col = nlte.Column(ctx, CASES["tiny"]())
    with pytest.raises(nlte.NLTEError) as e:
        col.solve(jv_method=5)
    assert e.value.status == nlte.NLTE_E_INVALID
