"""Edge cases at the limits of the library's sizes, against the FP64 oracle.

- the smallest column the library accepts: 3 depths, one angle per
  hemisphere, a few points per window (both formal-solution variants);
- the two-level atom (one line, no continuum transitions);
- the largest atom (16 levels, 24 lines and 15 edges; the preconditioner
  blocks are 16 x 16);
- sizes beyond the limits (17 levels, 9 angles, a depth-parallel column of
  257 depths, an empty batch) are rejected with NLTE_E_INVALID."""
import ctypes

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


def _parity(ctx, prob, precision, seed, want_P=True):
    from paper_2406_17234_amd import nlte
    tb = O.setup(prob)
    n = perturbed(tb.nstar, seed=seed, scale=0.2)
    ref = O.residual(tb, n, want_P=want_P)
    col = nlte.Column(ctx, prob, precision=precision)
    out = col.residual(to_dev(n), want_J=True, want_R=True, want_P=want_P)
    assert maxrel(to_np(out["J"]), ref.J, floor=1e-300) < 1e-11
    assert maxrel(to_np(out["R"])[..., 0], ref.R_lu, floor=1e-300) < 1e-11
    assert np.max(np.abs(to_np(out["F"]) - ref.F) / ref.G) < 1e-11
    if want_P:
        P = to_np(out["P"])
        for k in range(tb.nz):
            assert np.max(np.abs(P[k] - ref.P[k])) <= 1e-10 * np.max(np.abs(ref.P[k])), k
    col.close()


@pytest.mark.parametrize("scan", [False, True])
def test_smallest_column(ctx, scan):
    from paper_2406_17234_amd import nlte
    prob = S.tiny(nz=3, nmu=1, nline_pts=3, nbf_pts=2)
    print(f"[case] smallest column scan={scan} dims={prob.dims}", flush=True)
    _parity(ctx, prob, nlte.FP64 | (nlte.DEPTH_SCAN if scan else 0), seed=51)


def test_two_level_atom(ctx):
    from paper_2406_17234_amd import nlte
    prob = S.two_level(1e-2)
    print(f"[case] two-level dims={prob.dims}", flush=True)
    _parity(ctx, prob, nlte.FP64, seed=52)
    tb = O.setup(prob)
    ref = O.solve(tb, ftol=1e-12, rtol=1e-6, maxiter=60)
    assert ref.converged
    col = nlte.Column(ctx, prob, precision=nlte.FP64)
    n, _, st, rc = col.solve(ftol=1e-12, rtol=1e-6, maxiter=60)
    assert rc == 0 and st["rho_inf"] <= 1e-12
    assert maxrel(to_np(n), ref.n) < 1e-10


@pytest.mark.parametrize("nz", [8, 9, 10, 16, 17, 25])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("newton", [False, True])
def test_rate_blocks_at_every_depth_alignment(ctx, nz, precision, newton):
    """The formal-solution kernel integrates the rates in blocks of 8 depths
    per sweep and writes J through the same tile: columns whose depth count
    ends anywhere in a block (the bottom depth opening a block, ending one,
    or inside one) give the oracle's J, R and F in both modes."""
    from paper_2406_17234_amd import nlte
    prob = S.chromo6(nz=nz, nnu=150)
    tb = O.setup(prob)
    n = perturbed(tb.nstar, seed=nz, scale=0.2)
    ref = O.residual(tb, n)
    prec = nlte.FP64 if precision == "fp64" else nlte.FP32_FORM
    col = nlte.Column(ctx, prob, precision=prec)
    out = col.residual(to_dev(n), want_J=True, want_R=True, want_P=newton)
    tol = 1e-11 if precision == "fp64" else 5e-5
    big = ref.J > (1e-300 if precision == "fp64" else 1e-30 * ref.J.max())
    assert maxrel(to_np(out["J"])[big], ref.J[big]) < tol
    R = to_np(out["R"])
    assert maxrel(R[..., 0], ref.R_lu, floor=1e-300) < tol
    assert maxrel(R[..., 1], ref.R_ul, floor=1e-300) < tol
    assert np.max(np.abs(to_np(out["F"]) - ref.F) / ref.G) < 2 * tol
    col.close()


def _level_ladder(nlev, name):
    """An atom of nlev - 1 evenly spaced bound levels (0 to 7.5 eV) plus a
    continuum at 9 eV, lines between neighbours and next neighbours, an edge
    from every bound level."""
    nb = nlev - 1
    E_eV = np.concatenate([np.linspace(0.0, 7.5, nb), [9.0]])
    pairs = [(i, i + 1) for i in range(nb - 1)] + [(i, i + 2) for i in range(nb - 2)]
    pairs = pairs[:24]
    return S.Atom(name=name, E=E_eV * S.EV, g=np.array([2.0 + 2 * (i % 4) for i in range(nb)] + [1.0]),
                  stage=np.array([0] * nb + [1], np.int32),
                  line_lo=np.array([p[0] for p in pairs], np.int32),
                  line_up=np.array([p[1] for p in pairs], np.int32),
                  A_ul=np.full(len(pairs), 1e7), a_damp=np.full(len(pairs), 1e-3),
                  mass_amu=40.0, vturb=0.0, bf_lo=np.arange(nb, dtype=np.int32),
                  bf_alpha0=np.full(nb, 1e-18))


def _sixteen_levels():
    atom = _level_ladder(16, "ladder16")
    atm = S.chromosphere(nz=40, abund=2e-6, perturb_seed=61)
    nl, nb = S._split_points(500, atom.nline, atom.nbf)
    grid = S.make_grid(atom, atm, nl, nb, 3)
    return S.Problem("sixteen", atom, atm, grid, S.make_collisions(atom, atm), 61)


def test_largest_atom(ctx):
    from paper_2406_17234_amd import nlte
    prob = _sixteen_levels()
    print(f"[case] 16 levels dims={prob.dims}", flush=True)
    assert prob.atom.nlev == 16
    _parity(ctx, prob, nlte.FP64, seed=53)


def test_sizes_beyond_limits_rejected(ctx):
    from paper_2406_17234_amd import nlte
    big = S.tiny(nz=257, nmu=2)
    with pytest.raises(nlte.NLTEError) as e:
        nlte.Column(ctx, big, precision=nlte.FP64 | nlte.DEPTH_SCAN)
    assert e.value.status == nlte.NLTE_E_INVALID
    nlte.Column(ctx, big, precision=nlte.FP64).close()  # the sequential form has no depth limit
    with pytest.raises(nlte.NLTEError) as e:
        nlte.Column(ctx, S.tiny(nmu=9), precision=nlte.FP64)
    assert e.value.status == nlte.NLTE_E_INVALID
    atom = _level_ladder(17, "ladder17")
    atm = S.chromosphere(nz=20, abund=2e-6, perturb_seed=62)
    nl, nb = S._split_points(300, atom.nline, atom.nbf)
    p17 = S.Problem("seventeen", atom, atm, S.make_grid(atom, atm, nl, nb, 2),
                    S.make_collisions(atom, atm), 62)
    with pytest.raises(nlte.NLTEError) as e:
        nlte.Column(ctx, p17, precision=nlte.FP64)
    assert e.value.status == nlte.NLTE_E_INVALID
    # an empty batch
    L = nlte.lib()
    opts = nlte.default_opts()
    stats = (nlte.SolveStats * 1)()
    rc = L.nlte_solve_batch(ctx.h, None, 0, None, None, ctypes.byref(opts), None, stats, None)
    assert rc == nlte.NLTE_E_INVALID


def test_objects_outliving_their_context(ctx):
    """A column, plan or server destroyed after its context (as a cyclic
    garbage collection may order it) releases its memory on its own device
    and leaves no error behind for the next call."""
    from paper_2406_17234_amd import nlte
    other = nlte.Context(0)
    col = nlte.Column(other, S.tiny(), precision=nlte.FP64)
    tb = O.setup(S.tiny())
    nd = to_dev(tb.nstar)
    Fd = to_dev(np.zeros_like(tb.nstar))
    plan = nlte.Plan(other, [col], [nd], [Fd], graph=False)
    srv = nlte.Server(other, hbm_budget=1 << 30, max_active=4)
    other.close()
    srv.close()
    plan.close()
    col.close()
    fresh = nlte.Column(ctx, S.tiny(), precision=nlte.FP64)
    n = perturbed(tb.nstar, seed=54, scale=0.2)
    out = fresh.residual(to_dev(n))
    ref = O.residual(tb, n)
    assert np.max(np.abs(to_np(out["F"]) - ref.F) / ref.G) < 1e-11
    fresh.close()
