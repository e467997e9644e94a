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


def test_problem_requests_allocate_at_admission(ctx):
    """Problem requests: the server creates each column when it admits the
    request within the budget and frees it when the request retires, so the
    bytes in flight never exceed the budget, device memory returns when the
    stream is done, and each result equals the same problem solved alone."""
    import torch
    from paper_2406_17234_amd import nlte
    probs = [S.stream_request(j, nz_max=96, nnu_max=500) for j in range(10)]
    sizes = [nlte.plan_bytes(p, nlte.FP32_FORM) for p in probs]
    budget = 2 * max(sizes)
    alone = []
    for p in probs:
        c = nlte.Column(ctx, p, precision=nlte.FP32_FORM)
        n, _, st, _ = c.solve(**OPTS)
        alone.append((to_np(n), st))
        assert c.bytes == nlte.plan_bytes(p, nlte.FP32_FORM)
        c.close()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    srv = nlte.Server(ctx, hbm_budget=budget, max_active=64, **OPTS)
    outs = [torch.zeros(p.atmos.nz, p.atom.nlev, dtype=torch.float64, device="cuda") for p in probs]
    try:
        tickets = [srv.submit_problem(p, o, nlte.FP32_FORM) for p, o in zip(probs, outs)]
        lowest = free0
        res = {}
        t0 = time.time()
        while len(res) < len(tickets):
            lowest = min(lowest, torch.cuda.mem_get_info()[0])
            for t in tickets:
                if t not in res:
                    r = srv.poll(t)
                    if r is not None:
                        res[t] = r[1]
            assert time.time() - t0 < 300
            time.sleep(0.001)
        info = srv.info()
    finally:
        srv.close()
    torch.cuda.synchronize()
    assert info["peak_active_bytes"] <= budget
    # device memory held by the stream: the columns in flight (within the
    # budget) plus the server's work lists and solver buffers
    assert free0 - lowest <= budget + (64 << 20)
    assert torch.cuda.mem_get_info()[0] >= free0 - (64 << 20)
    for (na, sa), t, o in zip(alone, tickets, outs):
        r = res[t]
        assert r["status"] == sa["status"] and r["f_calls"] == sa["f_calls"]
        assert np.array_equal(to_np(o), na)
        assert r["t_submit_ms"] <= r["t_admit_ms"] <= r["t_done_ms"]


def test_invalid_problem_rejected_at_submission(ctx):
    import copy
    from paper_2406_17234_amd import nlte
    p = copy.deepcopy(S.slab3())
    p.atmos.T = p.atmos.T.copy()
    p.atmos.T[3] = np.nan
    import torch
    torch_out = torch.zeros(p.atmos.nz, p.atom.nlev, dtype=torch.float64, device="cuda")
    srv = nlte.Server(ctx, hbm_budget=1 << 30, max_active=4, **OPTS)
    try:
        with pytest.raises(nlte.NLTEError) as e:
            srv.submit_problem(p, torch_out)
        assert e.value.status == nlte.NLTE_E_NONFINITE
        assert srv.info()["submitted"] == 0
    finally:
        srv.close()


def test_radiation_free_start_served(ctx):
    """Served requests started from the radiation-free populations (opts.init
    = 2, Sect. 2.2.1) equal the batch solve with the same start."""
    from paper_2406_17234_amd import nlte
    opts = dict(OPTS, init=2, maxiter=6)
    probs = [S.slab3(), S.stream_request(2, nz_max=96, nnu_max=500)]
    cols = [nlte.Column(ctx, p, precision=nlte.FP64) for p in probs]
    ref, st_ref, _ = nlte.solve_batch(ctx, cols, **opts)
    srv = nlte.Server(ctx, hbm_budget=1 << 36, max_active=8, **opts)
    try:
        got = [_wait(srv, srv.submit(c), c) for c in cols]
    finally:
        srv.close()
    for (n, r), o, s in zip(got, ref, st_ref):
        assert r["f_calls"] == s["f_calls"]
        assert np.array_equal(n, to_np(o))


def test_full_size_eleven_level_request_alone_and_in_the_mix(ctx):
    """A full-size 11-level request (211 depths, 1800 frequencies, 6 angles)
    served among smaller ones gives the same result as alone."""
    from paper_2406_17234_amd import nlte
    big = S.stream_request(3)
    assert big.atom.nlev == 11 and big.atmos.nz > 200 and big.grid.nnu >= 1500
    print(f"[case] served 11-level dims={big.dims}", flush=True)
    opts = dict(OPTS, maxiter=20, max_krylov_total=200, fp64_fallback=12)
    cols = [nlte.Column(ctx, big, precision=nlte.FP32_FORM)] + _mixed_columns(ctx)[3:6]
    alone = [c.solve(**opts) for c in cols]
    srv = nlte.Server(ctx, hbm_budget=1 << 36, max_active=16, **opts)
    try:
        tickets = [srv.submit(c) for c in cols]
        got = [_wait(srv, t, c) for t, c in zip(tickets, cols)]
    finally:
        srv.close()
    for (n, _, sa, _), (ns, rs) in zip(alone, got):
        assert rs["status"] == sa["status"] and rs["f_calls"] == sa["f_calls"]
        assert np.array_equal(to_np(n), ns)
