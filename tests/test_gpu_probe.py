"""Issue-rate probes (the denominators of the depth recursion's VALU
roofline): each returns a plausible rate for a full device, and invalid
arguments are rejected."""
import pytest

from tests.helpers import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_2406_17234_amd import nlte
    return nlte.Context(0)


def test_issue_rates(ctx):
    """FP32 and FP64 FMAs issue between 1e12 and 1e15 lane operations per
    second on a full device; the exponential and the reciprocal, which run
    on the transcendental unit, are no faster than an FMA."""
    from paper_2406_17234_amd import nlte
    r = {op: ctx.issue_rate(op, 4096) for op in (nlte.PROBE_FMA_F32, nlte.PROBE_FMA_F64,
                                                 nlte.PROBE_EXP_F32, nlte.PROBE_RCP_F32)}
    print({k: f"{v:.3e}" for k, v in r.items()}, flush=True)
    for v in r.values():
        assert 1e11 < v < 1e15
    assert r[nlte.PROBE_FMA_F32] > 1e12 and r[nlte.PROBE_FMA_F64] > 1e12
    assert r[nlte.PROBE_EXP_F32] <= 1.05 * r[nlte.PROBE_FMA_F32]
    assert r[nlte.PROBE_RCP_F32] <= 1.05 * r[nlte.PROBE_FMA_F32]


def test_issue_rate_rejects_bad_arguments(ctx):
    from paper_2406_17234_amd import nlte
    for op, iters in ((4, 4096), (-1, 4096), (0, 0), (0, 4098), (0, 1 << 25)):
        with pytest.raises(nlte.NLTEError) as e:
            ctx.issue_rate(op, iters)
        assert e.value.status == nlte.NLTE_E_INVALID
