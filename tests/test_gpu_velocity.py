"""Velocity fields on the device (Sect. 3.5) against the FP64 oracle, in FP64
and in the FP32 form.

Each ray sees the line profiles Doppler-shifted by the velocity along it, so
the device builds the opacity ray by ray inside its formal solution, keeps
every ray's intensity for the line rates and every ray's local intensity
derivatives for the preconditioner.  Checked here: F, J, rates, Jbar and the
preconditioner blocks at 1 to 8 angles, the forward-difference product, roots
(GMRES and BiCGSTAB, and the full-size velocity-step column of the paper's
test against its stored oracle root), tangent (complex-step) products and
solves, a zero velocity field against the static column, batches and served
requests that mix static and velocity columns (each column bit for bit as
alone), and the combinations the library rejects."""
import copy

import numpy as np
import pytest

from oracle import nlte_oracle as O
from paper_2406_17234_amd import synth as S
from tests.golden.make_roots import load as load_root
from tests.helpers import maxrel, perturbed, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_2406_17234_amd import nlte
    return nlte.Context(0)


def _tiny_flow():
    p = copy.deepcopy(S.tiny())
    p.atmos.vlos = np.linspace(3e5, -2e5, p.atmos.nz)
    return p


PROBLEMS = {
    "tiny_flow": _tiny_flow,
    "vel_1mu": lambda: S.chromo6_vel(nz=17, nnu=160, nmu=1),
    "vel_small": lambda: S.chromo6_vel(nz=40, nnu=300, nmu=3),
    "vel_8mu": lambda: S.chromo6_vel(nz=25, nnu=200, nmu=8),
    "vel_full": S.chromo6_vel,
}


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_residual_matches_oracle(ctx, name):
    from paper_2406_17234_amd import nlte
    p = PROBLEMS[name]()
    tb = O.setup(p)
    assert tb.vel
    n = perturbed(tb.nstar, seed=5, scale=0.2)
    ref = O.residual(tb, n, want_P=True)
    print(f"[case] velocity residual {name} dims={p.dims}", flush=True)
    col = nlte.Column(ctx, p, precision=nlte.FP64)
    out = col.residual(to_dev(n), want_J=True, want_R=True, want_Jbar=True, want_P=True)
    # the device sums each line rate frequency by frequency over the rays,
    # the oracle ray by ray over the frequencies: F rows that cancel to 1e-4
    # of their gross rate G keep ~1e-12 G of the different rounding
    assert np.max(np.abs(to_np(out["F"]) - ref.F) / ref.G) < 5e-12
    J = to_np(out["J"])
    rel = np.abs(J - ref.J) / ref.J
    k, f = np.unravel_index(np.argmax(rel), rel.shape)
    print(f"J max rel {rel[k, f]:.2e} at k={k} f={f} J/Jmax={ref.J[k, f] / ref.J.max():.1e}", flush=True)
    assert rel.max() < 1e-10
    R = to_np(out["R"])
    assert maxrel(R[..., 0], ref.R_lu, floor=1e-300) < 1e-10
    assert maxrel(R[..., 1], ref.R_ul, floor=1e-300) < 1e-10
    assert maxrel(to_np(out["Jbar"]), ref.Jbar) < 1e-10
    P = to_np(out["P"])
    for k in range(tb.nz):
        assert np.max(np.abs(P[k] - ref.P[k])) <= 1e-10 * np.max(np.abs(ref.P[k])), k
    col.close()


def test_zero_velocity_equals_static_column(ctx):
    """A velocity field of zeros runs the ray-by-ray kernels and returns the
    static column's F and preconditioner to rounding."""
    from paper_2406_17234_amd import nlte
    p = S.chromo6(nz=40, nnu=300, nmu=3)
    q = copy.deepcopy(p)
    q.atmos.vlos = np.zeros(p.atmos.nz)
    tb = O.setup(p)
    n = perturbed(tb.nstar, seed=6, scale=0.2)
    a = nlte.Column(ctx, p, precision=nlte.FP64).residual(to_dev(n), want_P=True)
    b = nlte.Column(ctx, q, precision=nlte.FP64).residual(to_dev(n), want_P=True)
    G = O.residual(tb, n).G
    assert np.max(np.abs(to_np(a["F"]) - to_np(b["F"])) / G) < 1e-13
    Pa, Pb = to_np(a["P"]), to_np(b["P"])
    assert np.max(np.abs(Pa - Pb)) <= 1e-12 * np.max(np.abs(Pa))


def test_jvp_matches_oracle(ctx):
    from paper_2406_17234_amd import nlte
    p = PROBLEMS["vel_small"]()
    tb = O.setup(p)
    n = perturbed(tb.nstar, seed=3, scale=0.2)
    rng = np.random.default_rng(4)
    v = n * rng.standard_normal(n.shape)
    eps = 1e-7
    r0 = O.residual(tb, n)
    ref = O.jvp_fd(tb, n, v, r0.F, eps, rows=r0.rows)
    col = nlte.Column(ctx, p, precision=nlte.FP64)
    Jv = to_np(col.jvp(to_dev(n), to_dev(v), eps))
    # rounding of F (~1e-16 G) is amplified by 1/eps in both products
    assert np.max(np.abs(Jv - ref) / (r0.G / eps)) < 1e-12


_ROOT = {}


def _small_root():
    if "small" not in _ROOT:
        tb = O.setup(PROBLEMS["vel_small"]())
        s = O.solve(tb, ftol=1e-12, rtol=1e-6, maxiter=60)
        assert s.converged
        _ROOT["small"] = s
    return _ROOT["small"]


@pytest.mark.parametrize("method", ["gmres", "bicgstab"])
def test_solve_matches_oracle_root(ctx, method):
    from paper_2406_17234_amd import nlte
    ref = _small_root()
    km = nlte.KRYLOV_GMRES if method == "gmres" else nlte.KRYLOV_BICGSTAB
    print(f"[case] velocity solve {method}", flush=True)
    col = nlte.Column(ctx, PROBLEMS["vel_small"](), precision=nlte.FP64)
    n, J, st, rc = col.solve(ftol=1e-12, rtol=1e-6, maxiter=60, krylov_method=km, want_J=True)
    print(st, flush=True)
    assert rc == 0 and st["status"] == 0
    assert maxrel(to_np(n), ref.n) < 1e-10
    assert maxrel(to_np(J), ref.J, floor=1e-300) < 1e-9


def test_full_velocity_step_column_root(ctx):
    """The velocity-step column of the paper's velocity test (6-level atom,
    82 depths optimised for the gradient, 835 frequencies, 5 angles), solved
    from LTE with a Krylov tolerance of 1e-2, reaches the stored oracle root."""
    from paper_2406_17234_amd import nlte
    ref = load_root("chromo6_vel_root")
    p = S.chromo6_vel()
    assert ref.shape == (p.atmos.nz, p.atom.nlev)
    print(f"[case] velocity full root dims={p.dims}", flush=True)
    col = nlte.Column(ctx, p, precision=nlte.FP64)
    n, _, st, rc = col.solve(ftol=1e-12, rtol=1e-2, maxiter=80)
    print(st, flush=True)
    assert rc == 0 and st["status"] == 0
    assert maxrel(to_np(n), ref) < 1e-10


def test_mixed_batch_equals_alone(ctx):
    """Static and velocity columns solved in one batch, with forward-
    difference and with tangent products: each result and its counters
    equal the column solved alone, bit for bit."""
    from paper_2406_17234_amd import nlte
    specs = [(PROBLEMS["vel_small"](), nlte.FP64), (S.chromo6(nz=40, nnu=300), nlte.FP64),
             (_tiny_flow(), nlte.FP64), (S.slab3(), nlte.FP32_FORM),
             (PROBLEMS["vel_8mu"](), nlte.FP64), (PROBLEMS["vel_small"](), nlte.FP32_FORM)]
    cols = [nlte.Column(ctx, p, precision=pr) for p, pr in specs]
    for jv in (nlte.JV_FD, nlte.JV_TANGENT):
        opts = dict(ftol=1e-6, rtol=1e-4, maxiter=60, jv_method=jv, fp64_fallback=12)
        alone = [c.solve(**opts) for c in cols]
        outs, stats, rc = nlte.solve_batch(ctx, cols, **opts)
        for (n, _, sa, _), o, sb in zip(alone, outs, stats):
            assert sa["status"] == sb["status"] and sa["f_calls"] == sb["f_calls"]
            assert np.array_equal(to_np(n), to_np(o))


def test_served_velocity_request_equals_alone(ctx):
    import time

    import torch
    from paper_2406_17234_amd import nlte
    opts = dict(ftol=1e-10, rtol=1e-4, maxiter=60)
    probs = [PROBLEMS["vel_small"](), S.chromo6(nz=40, nnu=300), _tiny_flow()]
    alone = [nlte.Column(ctx, p, precision=nlte.FP64).solve(**opts) for p in probs]
    srv = nlte.Server(ctx, hbm_budget=1 << 34, max_active=8, **opts)
    outs = [torch.zeros(p.atmos.nz, p.atom.nlev, dtype=torch.float64, device="cuda") for p in probs]
    try:
        tickets = [srv.submit_problem(p, o, nlte.FP64) for p, o in zip(probs, outs)]
        res = {}
        t0 = time.time()
        while len(res) < len(tickets):
            for t in tickets:
                if t not in res:
                    r = srv.poll(t)
                    if r is not None:
                        res[t] = r[1]
            assert time.time() - t0 < 120
            time.sleep(0.002)
    finally:
        srv.close()
    for (n, _, sa, _), t, o in zip(alone, tickets, outs):
        assert res[t]["status"] == sa["status"] and res[t]["f_calls"] == sa["f_calls"]
        assert np.array_equal(to_np(o), to_np(n))


@pytest.mark.parametrize("name", ["tiny_flow", "vel_1mu", "vel_small", "vel_8mu"])
def test_tangent_product_matches_complex_step(ctx, name):
    """Tangent-linear products (the limit of Eq. complex) of velocity columns
    against the oracle's complex-step product through its ray-by-ray path."""
    from paper_2406_17234_amd import nlte
    p = PROBLEMS[name]()
    tb = O.setup(p)
    n = perturbed(tb.nstar, seed=71, scale=0.2)
    v = n * np.random.default_rng(72).standard_normal(n.shape)
    print(f"[case] velocity tangent product {name} dims={p.dims}", flush=True)
    ref = O.jvp_complex_step(tb, n, v)
    col = nlte.Column(ctx, p, precision=nlte.FP64)
    Jv = to_np(col.jvp_tangent(to_dev(n), to_dev(v)))
    err = np.max(np.abs(Jv - ref)) / np.max(np.abs(ref))
    print(f"  max err / max |Jv| = {err:.3e}", flush=True)
    assert err < 1e-12
    rows = O.conservation_rows(n)
    k = np.arange(tb.nz)
    assert np.allclose(Jv[k, rows], -v.sum(axis=1), rtol=1e-14, atol=0)
    col.close()


@pytest.mark.parametrize("method", ["gmres", "bicgstab"])
def test_tangent_solve_matches_oracle_root(ctx, method):
    """JFNK with exact (tangent) products on a velocity column reaches the
    oracle root, as the paper's complex-step solves do."""
    from paper_2406_17234_amd import nlte
    ref = _small_root()
    km = nlte.KRYLOV_GMRES if method == "gmres" else nlte.KRYLOV_BICGSTAB
    print(f"[case] velocity tangent solve {method}", flush=True)
    col = nlte.Column(ctx, PROBLEMS["vel_small"](), precision=nlte.FP64)
    n, _, st, rc = col.solve(ftol=1e-12, rtol=1e-6, maxiter=60, krylov_method=km,
                             jv_method=nlte.JV_TANGENT)
    print(st, flush=True)
    assert rc == 0 and st["status"] == 0
    assert maxrel(to_np(n), ref.n) < 1e-10


@pytest.mark.parametrize("name", ["vel_1mu", "vel_small", "vel_full"])
def test_fp32_form_residual(ctx, name):
    """The FP32 form (recursion in FP32, opacity sums, rates and F in FP64)
    of velocity columns against the FP64 oracle."""
    from paper_2406_17234_amd import nlte
    p = PROBLEMS[name]()
    tb = O.setup(p)
    n = perturbed(tb.nstar, seed=15, scale=0.2)
    ref = O.residual(tb, n)
    print(f"[case] velocity FP32 residual {name} dims={p.dims}", flush=True)
    col = nlte.Column(ctx, p, precision=nlte.FP32_FORM)
    out = col.residual(to_dev(n), want_J=True, want_R=True, want_Jbar=True)
    big = ref.J > 1e-30 * ref.J.max()
    assert maxrel(to_np(out["J"])[big], ref.J[big]) < 1e-4
    R = to_np(out["R"])
    assert maxrel(R[..., 0], ref.R_lu, floor=1e-300) < 1e-4
    assert maxrel(R[..., 1], ref.R_ul, floor=1e-300) < 1e-4
    assert maxrel(to_np(out["Jbar"]), ref.Jbar) < 1e-4
    assert np.max(np.abs(to_np(out["F"]) - ref.F) / ref.G) < 2e-4
    col.close()


def test_fp32_form_solve_within_1e4(ctx):
    """FP32-form velocity columns converge to within 1e-4 of the oracle's
    FP64 root (with the FP64 fallback enabled, as in the batch)."""
    from paper_2406_17234_amd import nlte
    ref = _small_root()
    col = nlte.Column(ctx, PROBLEMS["vel_small"](), precision=nlte.FP32_FORM)
    n, _, st, rc = col.solve(ftol=1e-6, rtol=1e-3, maxiter=60, fp64_fallback=12)
    print(st, flush=True)
    assert rc == 0 and st["status"] == 0
    assert maxrel(to_np(n), ref.n) < 1e-4
    full = load_root("chromo6_vel_root")
    col = nlte.Column(ctx, S.chromo6_vel(), precision=nlte.FP32_FORM)
    n, _, st, rc = col.solve(ftol=1e-6, rtol=1e-2, maxiter=80, fp64_fallback=12)
    print(st, flush=True)
    assert rc == 0 and st["status"] == 0
    assert maxrel(to_np(n), full) < 1e-4


def test_rejected_combinations(ctx):
    """Velocity columns: no depth-parallel variant."""
    from paper_2406_17234_amd import nlte
    p = _tiny_flow()
    for prec in (nlte.FP64 | nlte.DEPTH_SCAN, nlte.FP32_FORM | nlte.DEPTH_SCAN):
        with pytest.raises(nlte.NLTEError) as e:
            nlte.Column(ctx, p, precision=prec)
        assert e.value.status == nlte.NLTE_E_INVALID
    # a rejected creation leaves nothing behind: a valid column still works
    col = nlte.Column(ctx, p, precision=nlte.FP64)
    tb = O.setup(p)
    out = col.residual(to_dev(tb.nstar))
    assert np.all(np.isfinite(to_np(out["F"])))
