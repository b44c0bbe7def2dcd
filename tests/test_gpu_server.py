"""Served jobs (continuous batching under an HBM budget) through the C ABI:
every served result equals the oracle's partition of that job alone."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1402_3281_amd as sc

    sc.load_library()
    return sc


@pytest.fixture(scope="module")
def ctx(sc):
    c = sc.Context(0)
    yield c
    c.close()


def test_served_equals_alone(sc, ctx):
    specs = graphgen.serve_specs(count=10, seed=21, lg_lo=9, lg_hi=14)
    graphs = [s.make() for s in specs]
    devs = [sc.DeviceGraph.from_host(g) for g in graphs]
    parts = [torch.full((g.n,), -1, dtype=torch.int32, device="cuda") for g in graphs]
    # a budget of about two of the largest jobs, so that admission (and the
    # submission of input copies) waits for retirements
    budget = 2 * max(sc.server_footprint(g.n, g.m, s.k)[1] for g, s in zip(graphs, specs))
    srv = sc.Server(ctx, hbm_budget_bytes=budget, max_active=8)
    try:
        tickets = [srv.submit(d, s.k, p) for d, s, p in zip(devs, specs, parts)]
        del devs  # the server holds its own copies of the inputs
        results = [srv.wait(t) for t in tickets]
        for g, s, p, r in zip(graphs, specs, parts, results):
            assert r["status"] == sc.OK, g.name
            want_part, want = oracle.partition(g, s.k)
            got = p.cpu().numpy()
            assert np.array_equal(got, want_part), g.name
            assert r["cut"] == want["cut"] and r["max_block"] == want["max_block"], g.name
            assert r["latency_ms"] >= r["queue_ms"] >= 0.0
        st = srv.stats()
        assert st["completed"] == len(specs)
        assert 0 < st["peak_bytes"] <= budget
        assert st["p99_ms"] >= st["p50_ms"] > 0.0 and st["jobs_per_s"] > 0.0
    finally:
        srv.close()


def test_poll_and_unknown_ticket(sc, ctx):
    g = graphgen.rmat(11, 8, seed=31)
    d = sc.DeviceGraph.from_host(g)
    p = torch.empty(g.n, dtype=torch.int32, device="cuda")
    srv = sc.Server(ctx, hbm_budget_bytes=1 << 30)
    try:
        t = srv.submit(d, 8, p)
        r = srv.wait(t)
        assert r["status"] == sc.OK
        want_part, want = oracle.partition(g, 8)
        assert np.array_equal(p.cpu().numpy(), want_part) and r["cut"] == want["cut"]
        with pytest.raises(sc.SclapError):
            srv.poll(t)  # already taken
        with pytest.raises(sc.SclapError):
            srv.poll(t + 1000)
        t2 = srv.submit(d, 4, p)
        r2 = None
        while r2 is None:
            r2 = srv.poll(t2)
        assert r2["status"] == sc.OK
        want_part, want = oracle.partition(g, 4)
        assert np.array_equal(p.cpu().numpy(), want_part)
    finally:
        srv.close()


def test_budget_rejects_oversized_job(sc, ctx):
    g = graphgen.rmat(12, 8, seed=41)
    d = sc.DeviceGraph.from_host(g)
    p = torch.empty(g.n, dtype=torch.int32, device="cuda")
    srv = sc.Server(ctx, hbm_budget_bytes=1 << 16)
    try:
        with pytest.raises(sc.SclapError) as e:
            srv.submit(d, 4, p)
        assert e.value.code == sc.EBUDGET
    finally:
        srv.close()


def test_budget_of_one_job_runs_them_in_turn(sc, ctx):
    """A budget that holds the largest job and little else: submissions wait
    while the queued input copies would not fit, every job still completes,
    and each equals the oracle's partition of it alone."""
    specs = graphgen.serve_specs(count=6, seed=27, lg_lo=9, lg_hi=13)
    graphs = [s.make() for s in specs]
    devs = [sc.DeviceGraph.from_host(g) for g in graphs]
    parts = [torch.full((g.n,), -1, dtype=torch.int32, device="cuda") for g in graphs]
    budget = max(sc.server_footprint(g.n, g.m, s.k)[1] for g, s in zip(graphs, specs)) + 4096
    srv = sc.Server(ctx, hbm_budget_bytes=budget, max_active=4)
    try:
        tickets = [srv.submit(d, s.k, p) for d, s, p in zip(devs, specs, parts)]
        results = [srv.wait(t) for t in tickets]
        for g, s, p, r in zip(graphs, specs, parts, results):
            assert r["status"] == sc.OK, g.name
            want_part, want = oracle.partition(g, s.k)
            assert np.array_equal(p.cpu().numpy(), want_part), g.name
            assert r["cut"] == want["cut"], g.name
        assert srv.stats()["peak_bytes"] <= budget
    finally:
        srv.close()
