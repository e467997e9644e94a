"""GPU JFNK solves against the FP64 oracle's converged populations.

FP64 solves on both sides are driven to a scaled residual of 1e-14 (one
quadratic step past 1e-12, where a stop can leave ~1e-10 of the last
correction in the populations), so the Newton paths (which need not agree) no
longer matter; converged populations and profile-averaged intensities must
agree to 1e-10 relative (FP64) and 1e-4 (FP32 formal-solution form)."""
import numpy as np
import pytest

from oracle import nlte_oracle as O
from paper_2406_17234_amd import synth as S
from tests.helpers import maxrel, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu

_ORACLE_CACHE = {}


def oracle_root(name, maker, ftol=1e-14):
    if name not in _ORACLE_CACHE:
        prob = maker()
        tb = O.setup(prob)
        s = O.solve(tb, ftol=ftol, rtol=1e-6, maxiter=60)
        assert s.converged
        _ORACLE_CACHE[name] = (prob, tb, s)
    return _ORACLE_CACHE[name]


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_2406_17234_amd import nlte
    return nlte.Context(0)


CASES = {
    "tiny": lambda: S.tiny(),
    "slab3": lambda: S.slab3(),
    "chromo6_small": lambda: S.chromo6(nz=40, nnu=300),
    "chromo6": lambda: S.chromo6(),
}


@pytest.mark.parametrize("name", list(CASES))
def test_solve_fp64_matches_oracle_root(ctx, name):
    from paper_2406_17234_amd import nlte
    prob, tb, ref = oracle_root(name, CASES[name])
    print(f"[case] solve fp64 {name} dims={prob.dims}", flush=True)
    col = nlte.Column(ctx, prob)
    n, J, st, rc = col.solve(ftol=1e-14, rtol=1e-6, maxiter=60, want_J=True)
    print(st, flush=True)
    assert rc == 0 and st["status"] == 0
    assert st["rho_inf"] <= 1e-14
    n = to_np(n)
    assert maxrel(n, ref.n) < 1e-10
    out = col.residual(to_dev(n), want_Jbar=True)
    if tb.nline:
        rr = O.residual(tb, ref.n)
        assert maxrel(to_np(out["Jbar"])[:, :tb.nline], rr.Jbar) < 1e-10
    # particle conservation
    assert np.max(np.abs(n.sum(axis=1) / tb.ntot - 1)) < 1e-13


def test_solve_default_stop(ctx):
    """The default stop (scaled residual 1e-8) on the 3-level slab."""
    from paper_2406_17234_amd import nlte
    prob, tb, ref = oracle_root("slab3", CASES["slab3"])
    col = nlte.Column(ctx, prob)
    n, _, st, rc = col.solve(ftol=1e-8)
    assert rc == 0 and st["rho_inf"] <= 1e-8
    assert maxrel(to_np(n), ref.n) < 1e-5


def test_zero_radiation_guess(ctx):
    from paper_2406_17234_amd import nlte
    prob = CASES["chromo6_small"]()
    tb = O.setup(prob)
    ref = O.zero_radiation_guess(tb)
    col = nlte.Column(ctx, prob)
    # a dense per-depth solve over ~16 decades of populations: FP64 parity bar
    assert maxrel(to_np(col.zero_radiation()), ref) < 1e-10
    # this guess is poor for the synthetic 6-level atom (the oracle does not
    # converge from it either); the solve must still end cleanly
    n, _, st, rc = col.solve(init=2, ftol=1e-10, rtol=1e-4, maxiter=5)
    assert rc in (0, nlte.NLTE_E_NOCONV) and st["newton_iters"] <= 5
    assert np.all(np.isfinite(to_np(n)))


def test_batch_equals_single(ctx):
    """A column solved inside a batch gives bit-identical populations to the
    same column solved alone."""
    from paper_2406_17234_amd import nlte
    probs = [CASES["slab3"](), CASES["chromo6_small"](), CASES["tiny"]()]
    cols = [nlte.Column(ctx, p) for p in probs]
    outs, stats, rc = nlte.solve_batch(ctx, cols, ftol=1e-10, rtol=1e-4)
    assert rc == 0, stats
    for c, o in zip(cols, outs):
        n1, _, st, rc1 = c.solve(ftol=1e-10, rtol=1e-4)
        assert rc1 == 0
        assert np.array_equal(to_np(n1), to_np(o))


def test_batch_with_every_launch_list_equals_alone(ctx):
    """Each step sorts the columns' chunks into the lists of the launches
    that evaluate them (F or Newton mode, in the FP32 form or in FP64 after
    a fallback).  A batch whose FP32-form columns fall back to FP64 after two
    Newton iterations, beside FP64 columns, keeps all four lists busy at once
    and in changing mixes; every column must still get the populations and
    statistics it gets alone, bit for bit."""
    from paper_2406_17234_amd import nlte
    probs = ([S.batch6_column(i) for i in range(6)] +
             [S.stream_request(j, nz_max=96, nnu_max=500) for j in (0, 1, 5)] +
             [CASES["slab3"](), CASES["chromo6_small"]()])
    precs = [nlte.FP32_FORM] * 9 + [nlte.FP64] * 2
    cols = [nlte.Column(ctx, p, precision=pr) for p, pr in zip(probs, precs)]
    opts = dict(ftol=1e-8, rtol=1e-3, maxiter=30, max_krylov_total=300, fp64_fallback=2)
    print("[case] mixed batch, fallback after 2 iterations", flush=True)
    outs, stats, rc = nlte.solve_batch(ctx, cols, **opts)
    assert sum(s["precision"] == nlte.FP64 for s in stats[:9]) >= 3, stats
    for c, o, s in zip(cols, outs, stats):
        n1, _, s1, _ = c.solve(**opts)
        assert np.array_equal(to_np(n1), to_np(o))
        assert s1 == s


def test_fp32_form_within_1e4(ctx):
    from paper_2406_17234_amd import nlte
    prob, tb, ref = oracle_root("chromo6", CASES["chromo6"])
    col = nlte.Column(ctx, prob, precision=nlte.FP32_FORM)
    n, _, st, rc = col.solve(ftol=1e-6, rtol=1e-3, maxiter=60)
    print(st, flush=True)
    assert rc == 0
    assert maxrel(to_np(n), ref.n) < 1e-4


def test_maxiter_reports_noconv(ctx):
    from paper_2406_17234_amd import nlte
    prob = CASES["chromo6_small"]()
    col = nlte.Column(ctx, prob)
    n, _, st, rc = col.solve(ftol=1e-14, maxiter=1)
    assert rc == nlte.NLTE_E_NOCONV and st["status"] == nlte.NLTE_E_NOCONV
    assert st["newton_iters"] == 1
    assert np.all(np.isfinite(to_np(n)))


def test_krylov_cap_is_per_newton_step(ctx):
    """max_krylov bounds the Krylov iterations of each Newton step, not of the
    whole solve: a solve whose total exceeds the cap still converges."""
    from paper_2406_17234_amd import nlte
    prob, tb, ref = oracle_root("chromo6_small", CASES["chromo6_small"])
    col = nlte.Column(ctx, prob)
    n, _, st, rc = col.solve(ftol=1e-12, rtol=1e-6, maxiter=60, max_krylov=40)
    assert st["krylov_iters"] > 40
    assert rc == 0 and st["rho_inf"] <= 1e-12
    assert maxrel(to_np(n), ref.n) < 1e-10


def test_krylov_budget_per_solve(ctx):
    """Once max_krylov_total is spent every Newton iteration takes a single
    Krylov step."""
    from paper_2406_17234_amd import nlte
    prob = CASES["chromo6_small"]()
    col = nlte.Column(ctx, prob)
    n, _, st, rc = col.solve(ftol=1e-12, rtol=1e-6, maxiter=8, max_krylov_total=10)
    assert st["krylov_iters"] <= 10 + st["newton_iters"]
    assert st["newton_iters"] >= 1


def test_fp32_form_falls_back_to_fp64(ctx):
    """An 11-level FP32-form column that the FP32 formal solution cannot
    drive to convergence finishes in FP64 after the fallback, at the FP64
    root (to the FP32-form tolerance)."""
    from paper_2406_17234_amd import nlte
    prob = S.stream_request(0, nz_max=96, nnu_max=500)
    c64 = nlte.Column(ctx, prob, precision=nlte.FP64)
    n64, _, s64, rc64 = c64.solve(ftol=1e-6, rtol=1e-3, maxiter=40)
    assert rc64 == 0
    c32 = nlte.Column(ctx, prob, precision=nlte.FP32_FORM)
    n32, _, s32, rc32 = c32.solve(ftol=1e-6, rtol=1e-3, maxiter=40, fp64_fallback=10)
    print(s32, flush=True)
    assert rc32 == 0 and s32["precision"] == nlte.FP64 and s32["fp64_evals"] > 0
    assert maxrel(to_np(n32), to_np(n64)) < 1e-4
    # without the fallback the column stays in FP32 (and its stats say so)
    _, _, s0, _ = c32.solve(ftol=1e-6, rtol=1e-3, maxiter=3)
    assert s0["precision"] == nlte.FP32_FORM and s0["fp64_evals"] == 0


def test_fp64_fallback_keeps_a_close_iterate(ctx):
    """At the fallback an FP32-form iterate within max |F|/G <= 1e-2 of the
    root is kept (FP64 then needs only a few Newton iterations), while one
    further away starts again from LTE (as many FP64 iterations as a plain
    FP64 solve).  ftol = 1e-12 is out of the FP32 form's reach, so the
    fallback always triggers; both runs end at the FP64 root."""
    from paper_2406_17234_amd import nlte
    prob, tb, ref = oracle_root("chromo6_small", CASES["chromo6_small"])
    c64 = nlte.Column(ctx, prob, precision=nlte.FP64)
    _, _, s64, rc64 = c64.solve(ftol=1e-12, rtol=1e-6, maxiter=40)
    assert rc64 == 0
    c32 = nlte.Column(ctx, prob, precision=nlte.FP32_FORM)
    rho = {}
    for k in range(1, 13):
        _, _, sk, _ = c32.solve(ftol=1e-12, rtol=1e-6, maxiter=k)
        rho[k] = sk["rho_inf"]
    print(rho, s64, flush=True)
    far = [k for k in rho if rho[k] > 0.1]
    close = [k for k in rho if rho[k] <= 1e-3]
    assert far and close
    for k, kept in ((max(far), False), (min(close), True)):
        n, _, st, rc = c32.solve(ftol=1e-12, rtol=1e-6, maxiter=40, fp64_fallback=k)
        print(k, kept, st, flush=True)
        assert rc == 0 and st["precision"] == nlte.FP64
        assert maxrel(to_np(n), ref.n) < 1e-10
        fp64_its = st["newton_iters"] - k
        if kept:
            assert fp64_its < s64["newton_iters"]
        else:
            assert abs(fp64_its - s64["newton_iters"]) <= 1


@pytest.mark.parametrize("name", ["slab3", "chromo6_small"])
def test_bicgstab_fp64_matches_oracle_root(ctx, name):
    """JFNK with the BiCGSTAB inner solver (Sect. 2.3) reaches the oracle's
    root; both inner solvers converge to the same solution (Sect. 3.2)."""
    from paper_2406_17234_amd import nlte
    prob, tb, ref = oracle_root(name, CASES[name])
    col = nlte.Column(ctx, prob)
    n, _, st, rc = col.solve(ftol=1e-12, rtol=1e-6, maxiter=60,
                             krylov_method=nlte.KRYLOV_BICGSTAB)
    print(st, flush=True)
    assert rc == 0 and st["rho_inf"] <= 1e-12
    assert maxrel(to_np(n), ref.n) < 1e-10
    # two products with the Jacobian per BiCGSTAB iteration, one residual call each
    assert st["f_calls"] >= st["krylov_iters"] + st["newton_iters"]


def test_bicgstab_fp32_form_batch(ctx):
    """Batched FP32-form columns with BiCGSTAB converge to within 1e-4 of the
    FP64 root; the Krylov budget counts products."""
    from paper_2406_17234_amd import nlte
    prob, tb, ref = oracle_root("chromo6", CASES["chromo6"])
    cols = [nlte.Column(ctx, prob, precision=nlte.FP32_FORM) for _ in range(3)]
    outs, stats, rc = nlte.solve_batch(ctx, cols, ftol=1e-6, rtol=1e-3, maxiter=60,
                                       krylov_method=nlte.KRYLOV_BICGSTAB, fp64_fallback=30)
    assert rc == 0
    for o, s in zip(outs, stats):
        assert s["status"] == 0
        assert maxrel(to_np(o), ref.n) < 1e-4
    col = nlte.Column(ctx, CASES["chromo6_small"]())
    _, _, st, _ = col.solve(ftol=1e-12, rtol=1e-6, maxiter=8, max_krylov_total=10,
                            krylov_method=nlte.KRYLOV_BICGSTAB)
    assert st["krylov_iters"] <= 10 + st["newton_iters"]


def test_unknown_krylov_method_rejected(ctx):
    from paper_2406_17234_amd import nlte
    col = nlte.Column(ctx, CASES["tiny"]())
    with pytest.raises(nlte.NLTEError) as e:
        col.solve(krylov_method=7)
    assert e.value.status == nlte.NLTE_E_INVALID
