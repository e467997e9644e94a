"""Residual plans: F of several columns in shared launches, replayed from a
captured HIP graph.  Every replay must equal the eager evaluation bit for
bit, also with the program's own eager work and synchronisations between
replays and after the inputs change in place."""
import numpy as np
import pytest

from oracle import nlte_oracle as O
from paper_2406_17234_amd import synth as S
from tests.helpers import perturbed, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    require_gpu()
    import torch
    from paper_2406_17234_amd import nlte
    ctx = nlte.Context(0)
    probs = [(S.slab3(), nlte.FP64), (S.chromo6(nz=40, nnu=300), nlte.FP32_FORM),
             (S.chromo6(nz=40, nnu=300), nlte.FP64), (S.stream_request(2, nz_max=96, nnu_max=500), nlte.FP32_FORM)]
    cols = [nlte.Column(ctx, p, precision=prec) for p, prec in probs]
    ns = [to_dev(perturbed(O.setup(p).nstar, seed=11 + i, scale=0.2)) for i, (p, _) in enumerate(probs)]
    Fs = [torch.empty_like(n) for n in ns]
    return ctx, cols, ns, Fs


def _alone(cols, ns):
    return [to_np(c.residual(n)["F"]) for c, n in zip(cols, ns)]


def test_plan_equals_single_column_residual(setup):
    from paper_2406_17234_amd import nlte
    ctx, cols, ns, Fs = setup
    ref = _alone(cols, ns)
    plan = nlte.Plan(ctx, cols, ns, Fs, graph=False)
    plan.run()
    for a, b in zip(ref, Fs):
        assert np.array_equal(a, to_np(b))
    plan.close()


def test_graph_replays_match_eager(setup):
    import torch
    from paper_2406_17234_amd import nlte
    ctx, cols, ns, Fs = setup
    eager = nlte.Plan(ctx, cols, ns, [torch.empty_like(f) for f in Fs], graph=False)
    graph = nlte.Plan(ctx, cols, ns, Fs, graph=True)
    assert graph.info()["graph"] == 1
    for rep in range(4):
        if rep == 2:  # inputs change in place between replays
            for n in ns:
                n.mul_(1.01)
        eager.run()
        torch.cuda.synchronize()
        ref = [to_np(f) for f in eager._keep[2]]
        _ = cols[0].residual(ns[0])  # the program's own eager work in between
        graph.run()
        torch.cuda.synchronize()
        for a, b in zip(ref, Fs):
            assert np.array_equal(a, to_np(b)), rep
    eager.close()
    graph.close()


def test_tuned_plan(setup):
    from paper_2406_17234_amd import nlte
    ctx, cols, ns, Fs = setup
    ref = _alone(cols, ns)
    plan = nlte.Plan(ctx, cols, ns, Fs, graph=True, tune=True)
    info = plan.info()
    assert info["opac_depths"] in (4, 8, 16) and info["formal_wpb"] in (1, 2, 4)
    assert all(t > 0 for t in info["tune_ms"])
    plan.run()
    for a, b in zip(ref, Fs):
        assert np.array_equal(a, to_np(b))
    plan.close()
