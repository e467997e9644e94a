"""Batch solves whose step blocks are replayed from captured HIP graphs
(NLTE_SOLVE_GRAPH), with and without the launch-shape tuner
(NLTE_SOLVE_TUNE), against the eager launches: the populations and every
per-column statistic must be identical, bit for bit, over solves that replay
each graph many times with host synchronisations between replays and capture
again after every compaction of the running columns."""
import numpy as np
import pytest

from paper_2406_17234_amd import synth as S
from tests.helpers import require_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    require_gpu()
    from paper_2406_17234_amd import nlte
    ctx = nlte.Context(0)
    probs = ([S.batch6_column(i) for i in range(20)] +
             [S.stream_request(j, nz_max=96, nnu_max=500) for j in range(8)] + [S.slab3()])
    precs = [nlte.FP32_FORM] * 20 + [nlte.FP32_FORM] * 8 + [nlte.FP64]
    cols = [nlte.Column(ctx, p, precision=pr) for p, pr in zip(probs, precs)]
    return nlte, ctx, cols


def _solve(nlte, ctx, cols, launch):
    outs, stats, rc = nlte.solve_batch(ctx, cols, ftol=1e-6, rtol=1e-3, maxiter=40,
                                       max_krylov_total=200, fp64_fallback=12, launch=launch)
    return [to_np(o) for o in outs], stats, rc, ctx.read_profile()


def test_graph_replay_equals_eager(batch):
    nlte, ctx, cols = batch
    print("[case] graph solve vs eager", flush=True)
    ref, st_ref, rc_ref, _ = _solve(nlte, ctx, cols, 0)
    for launch in (nlte.NLTE_SOLVE_GRAPH, nlte.NLTE_SOLVE_GRAPH | nlte.NLTE_SOLVE_TUNE,
                   nlte.NLTE_SOLVE_GRAPH):
        outs, st, rc, prof = _solve(nlte, ctx, cols, launch)
        assert rc == rc_ref
        assert prof["last_graph"] == 1 and prof["last_captures"] >= 2
        for a, b in zip(outs, ref):
            assert np.array_equal(a, b)
        assert st == st_ref
        if launch & nlte.NLTE_SOLVE_TUNE:
            assert prof["last_formal_wpb"] in (1, 2, 4)
            assert all(t > 0 for t in prof["last_tune_ms"])
        else:
            assert prof["last_formal_wpb"] == 1


def test_tuned_eager_equals_eager(batch):
    nlte, ctx, cols = batch
    ref, st_ref, _, _ = _solve(nlte, ctx, cols, 0)
    outs, st, _, prof = _solve(nlte, ctx, cols, nlte.NLTE_SOLVE_TUNE)
    assert prof["last_graph"] == 0
    for a, b in zip(outs, ref):
        assert np.array_equal(a, b)
    assert st == st_ref


def test_profiled_solve_launches_eagerly(batch):
    nlte, ctx, cols = batch
    ctx.profile(True)
    try:
        _, _, _, prof = _solve(nlte, ctx, cols[:3], nlte.NLTE_SOLVE_GRAPH)
        assert prof["last_graph"] == 0 and prof["steps"] > 0
    finally:
        ctx.profile(False)


def test_bad_launch_flags_rejected(batch):
    nlte, ctx, cols = batch
    with pytest.raises(nlte.NLTEError) as e:
        nlte.solve_batch(ctx, cols[:1], launch=8)
    assert e.value.status == nlte.NLTE_E_INVALID
