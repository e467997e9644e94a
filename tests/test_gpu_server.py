"""Serving loop: continuous batching of column solves.

Each served result must equal the same column solved alone with the same
options (bit for bit: the per-column arithmetic does not depend on what else
is in flight), requests arriving while others run are admitted, and the HBM
budget bounds the device memory of the columns in flight."""
import time

import numpy as np
import pytest

from paper_2406_17234_amd import synth as S
from tests.helpers import require_gpu, to_np

pytestmark = pytest.mark.gpu

OPTS = dict(ftol=1e-6, rtol=1e-3, maxiter=40)


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_2406_17234_amd import nlte
    return nlte.Context(0)


def _mixed_columns(ctx):
    from paper_2406_17234_amd import nlte
    specs = [(S.slab3(), nlte.FP64), (S.chromo6(nz=40, nnu=300), nlte.FP32_FORM), (S.tiny(), nlte.FP64)]
    specs += [(S.stream_request(j, nz_max=96, nnu_max=500), nlte.FP32_FORM) for j in range(5)]
    return [nlte.Column(ctx, p, precision=prec) for p, prec in specs]


def _wait(srv, ticket, col, timeout=120.0):
    import torch
    out = torch.empty(col.nz, col.nlev, dtype=torch.float64, device=col.device)
    t0 = time.time()
    while True:
        r = srv.poll(ticket, out)
        if r is not None:
            return to_np(out), r[1]
        assert time.time() - t0 < timeout, "server did not finish in time"
        time.sleep(0.002)


@pytest.mark.parametrize("krylov,jv", [(0, 0), (1, 0), (0, 1)],
                         ids=["gmres", "bicgstab", "gmres-tangent"])
def test_served_equals_alone(ctx, krylov, jv):
    from paper_2406_17234_amd import nlte
    opts = dict(OPTS, krylov_method=krylov, jv_method=jv)
    cols = _mixed_columns(ctx)
    alone = []
    for c in cols:
        n, _, st, rc = c.solve(**opts)
        alone.append((to_np(n), st))
    srv = nlte.Server(ctx, hbm_budget=1 << 36, max_active=64, **opts)
    try:
        first = [srv.submit(c) for c in cols[:3]]
        n0, r0 = _wait(srv, first[0], cols[0])        # later requests arrive mid-flight
        rest = [srv.submit(c) for c in cols[3:]]
        got = [(n0, r0)] + [_wait(srv, t, c) for t, c in zip(first[1:] + rest, cols[1:])]
        srv.drain(60)
        info = srv.info()
    finally:
        srv.close()
    for (na, sa), (ns, rs) in zip(alone, got):
        assert rs["status"] == sa["status"]
        assert rs["newton_iters"] == sa["newton_iters"] and rs["f_calls"] == sa["f_calls"]
        assert np.array_equal(na, ns)
        assert rs["t_submit_ms"] <= rs["t_admit_ms"] <= rs["t_done_ms"]
    assert info["completed"] == len(cols) and info["active"] == 0 and info["queued"] == 0


def test_budget_bounds_columns_in_flight(ctx):
    from paper_2406_17234_amd import nlte
    cols = _mixed_columns(ctx)
    budget = max(c.bytes for c in cols) + min(c.bytes for c in cols)
    srv = nlte.Server(ctx, hbm_budget=budget, max_active=64, **OPTS)
    try:
        tickets = [srv.submit(c) for c in cols]
        res = [_wait(srv, t, c)[1] for t, c in zip(tickets, cols)]
    finally:
        srv.close()
    # at any admission instant, the columns in flight fit the budget
    for i, ri in enumerate(res):
        t = ri["t_admit_ms"]
        inflight = sum(c.bytes for c, r in zip(cols, res) if r["t_admit_ms"] <= t < r["t_done_ms"])
        assert inflight <= budget or inflight == cols[i].bytes
    print([r["status"] for r in res], flush=True)
    assert all(r["status"] != nlte.NLTE_E_DEVICE for r in res)


def test_poll_unknown_ticket(ctx):
    from paper_2406_17234_amd import nlte
    srv = nlte.Server(ctx, hbm_budget=1 << 30, max_active=4, **OPTS)
    try:
        with pytest.raises(nlte.NLTEError):
            srv.poll(12345)
    finally:
        srv.close()
