"""GPU parity of the residual path against the FP64 oracle, element by element
on the same seeded inputs: mean intensity J, radiative rates R, profile-
averaged line intensity Jbar, residual F (relative to the gross rates), the
block-Jacobi preconditioner P, and the forward-difference product Jv."""
import numpy as np
import pytest

from oracle import nlte_oracle as O
from paper_2406_17234_amd import synth as S
from tests.helpers import maxrel, perturbed, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu

PROBLEMS = {
    "tiny": lambda: S.tiny(),
    "slab3": lambda: S.slab3(),
    "chromo6_small": lambda: S.chromo6(nz=40, nnu=300),
    "chromo6": lambda: S.chromo6(),
}


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_2406_17234_amd import nlte
    return nlte.Context(0)


def _column(ctx, prob, prec=0):
    from paper_2406_17234_amd import nlte
    return nlte.Column(ctx, prob, precision=prec)


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_residual_fp64_matches_oracle(ctx, name):
    prob = PROBLEMS[name]()
    print(f"[case] residual fp64 {name} dims={prob.dims}", flush=True)
    tb = O.setup(prob)
    n = perturbed(tb.nstar, seed=1, scale=0.2)
    ref = O.residual(tb, n, want_P=True)
    col = _column(ctx, prob)
    out = col.residual(to_dev(n), want_J=True, want_R=True, want_Jbar=True, want_P=True)
    J = to_np(out["J"])
    assert maxrel(J, ref.J, floor=1e-300) < 1e-12
    R = to_np(out["R"])
    assert maxrel(R[..., 0], ref.R_lu, floor=1e-300) < 1e-12
    assert maxrel(R[..., 1], ref.R_ul) < 1e-12
    if tb.nline:
        assert maxrel(to_np(out["Jbar"])[:, :tb.nline], ref.Jbar) < 1e-12
    F = to_np(out["F"])
    assert np.max(np.abs(F - ref.F) / ref.G) < 1e-12
    P = to_np(out["P"])
    for k in range(tb.nz):
        assert np.max(np.abs(P[k] - ref.P[k])) <= 1e-11 * np.max(np.abs(ref.P[k])), k


@pytest.mark.parametrize("name", ["slab3", "chromo6_small"])
def test_residual_lte_planck_limit(ctx, name):
    """At LTE populations the device source function makes F small where the
    oracle's is small: compare the scaled residual vectors."""
    prob = PROBLEMS[name]()
    tb = O.setup(prob)
    ref = O.residual(tb, tb.nstar)
    col = _column(ctx, prob)
    n = col.lte()
    assert maxrel(to_np(n), tb.nstar) < 1e-13
    F = to_np(col.residual(n)["F"])
    assert np.max(np.abs(F - ref.F) / ref.G) < 1e-12


@pytest.mark.parametrize("name", ["slab3", "chromo6_small"])
def test_residual_fp32_form_close_to_oracle(ctx, name):
    prob = PROBLEMS[name]()
    print(f"[case] residual fp32 {name}", flush=True)
    tb = O.setup(prob)
    n = perturbed(tb.nstar, seed=2, scale=0.2)
    ref = O.residual(tb, n)
    col = _column(ctx, prob, prec=1)
    out = col.residual(to_dev(n), want_J=True, want_R=True, want_P=True)
    J = to_np(out["J"])
    big = ref.J > 1e-30 * ref.J.max()
    assert maxrel(J[big], ref.J[big]) < 5e-5
    R = to_np(out["R"])
    assert maxrel(R[..., 1], ref.R_ul) < 5e-5
    # preconditioner blocks from the FP32 recursion's derivatives
    refP = O.residual(tb, n, want_P=True).P
    P = to_np(out["P"])
    for k in range(tb.nz):
        assert np.max(np.abs(P[k] - refP[k])) <= 1e-4 * np.max(np.abs(refP[k])), k


def test_jvp_matches_oracle(ctx):
    prob = PROBLEMS["chromo6_small"]()
    tb = O.setup(prob)
    n = perturbed(tb.nstar, seed=3, scale=0.2)
    rng = np.random.default_rng(4)
    v = n * rng.standard_normal(n.shape)
    eps = 1e-7
    r0 = O.residual(tb, n)
    ref = O.jvp_fd(tb, n, v, r0.F, eps, rows=r0.rows)
    col = _column(ctx, prob)
    Jv = to_np(col.jvp(to_dev(n), to_dev(v), eps))
    # rounding of F (~1e-16 G) is amplified by 1/eps in both products
    assert np.max(np.abs(Jv - ref) / (r0.G / eps)) < 1e-12


def test_batched_tiles_independent_of_neighbours(ctx):
    """Two columns evaluated one after the other give bit-identical F to the
    same column evaluated alone (no cross-column state)."""
    p1 = PROBLEMS["chromo6_small"]()
    p2 = PROBLEMS["slab3"]()
    c1 = _column(ctx, p1)
    c2 = _column(ctx, p2)
    n1 = c1.lte()
    a = to_np(c1.residual(n1)["F"])
    c2.residual(c2.lte())
    b = to_np(c1.residual(n1)["F"])
    assert np.array_equal(a, b)


@pytest.mark.parametrize("name,prec", [("chromo6", 0), ("chromo6_small", 1)])
def test_f_only_and_newton_mode_agree_bitwise(ctx, name, prec):
    """The residual-only evaluation and the Newton-mode evaluation (which also
    builds the preconditioner) must give bit-identical F and J: the
    finite-difference product subtracts one from the other, so any rounding
    difference between the two would be amplified by 1/eps."""
    prob = PROBLEMS[name]()
    tb = O.setup(prob)
    n = perturbed(tb.nstar, seed=5, scale=0.2)
    col = _column(ctx, prob, prec)
    a = col.residual(to_dev(n), want_J=True)
    b = col.residual(to_dev(n), want_J=True, want_P=True)
    assert np.array_equal(to_np(a["F"]), to_np(b["F"]))
    assert np.array_equal(to_np(a["J"]), to_np(b["J"]))
