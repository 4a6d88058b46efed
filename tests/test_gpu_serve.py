"""Query server: continuous batching over several streams, HBM-budget
admission, and per-request results independent of the mix."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def server_parts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_15883_amd import serve
    boxes, thetas = wl.serving_nets(seed=2, width=24, depth=3)
    ctx = serve.serving_context(boxes, thetas, 24, 3, device="cuda")
    yield serve, ctx, boxes, thetas
    ctx.close()


def make_requests(serve, n_req, seed, nmax=5000, rate=2000.0):
    arr, sizes = wl.query_requests(seed, n_req, rate_hz=rate, nmax=nmax)
    rng = np.random.default_rng(seed)
    return [serve.Request(i, float(arr[i]), wl.query_points(rng, int(sizes[i]))) for i in range(n_req)]


def test_results_same_alone_and_in_mix(server_parts, orc):
    serve, ctx, boxes, thetas = server_parts
    reqs = make_requests(serve, 60, seed=4)
    srv = serve.QueryServer(ctx, hbm_budget_bytes=1 << 30, n_streams=3, max_batch_points=20000)
    srv.run(reqs)
    for r in reqs[:: 7]:
        alone = ctx.query(torch.from_numpy(r.x).cuda(), sub=-1, what="uvpw").cpu().numpy()
        np.testing.assert_array_equal(r.out, alone)
    # and against the oracle on a few requests
    for r in reqs[:3]:
        ref = orc.query2d(24, 3, thetas, boxes, r.x)
        err = np.abs(r.out[:, :3] - ref[:, :3]) / (np.abs(ref[:, :3]) + np.sqrt(np.mean(ref[:, :3] ** 2)))
        assert err.max() < 1e-5
    st = serve.latency_stats(reqs)
    assert st["p50_ms"] > 0 and st["p99_ms"] >= st["p50_ms"]


def test_small_budget_defers_without_error(server_parts):
    serve, ctx, _, _ = server_parts
    reqs = make_requests(serve, 40, seed=5, nmax=20000, rate=1e6)   # all arrive at once
    one = serve.QueryServer(ctx, n_streams=1, max_batch_points=20000)
    budget = 2 * one.slot_bytes
    del one
    srv = serve.QueryServer(ctx, hbm_budget_bytes=budget, n_streams=4, max_batch_points=20000)
    assert srv.n_slots == 2 and srv.device_bytes <= budget
    srv.run(reqs)
    assert srv.deferred > 0
    assert all(r.out is not None and r.out.shape == (len(r.x), 4) for r in reqs)


def test_16mb_budget_bounds_device_memory(server_parts):
    """Admission at a 16 MB HBM budget: the server's own device allocation
    stays within the budget while requests of up to 200,000 points are
    served (they wait for a free batch slot)."""
    serve, ctx, _, _ = server_parts
    budget = 16 << 20
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    srv = serve.QueryServer(ctx, hbm_budget_bytes=budget, n_streams=4, max_batch_points=200_000)
    held = torch.cuda.memory_allocated() - before
    assert held <= budget and srv.device_bytes <= budget
    assert 1 <= srv.n_slots < 4
    arr, sizes = wl.query_requests(8, 12, rate_hz=1e5, nmax=200_000)
    sizes[:3] = [200_000, 150_000, 1]
    rng = np.random.default_rng(8)
    reqs = [serve.Request(i, float(arr[i]), wl.query_points(rng, int(sizes[i]))) for i in range(12)]
    srv.run(reqs)
    assert torch.cuda.memory_allocated() - before <= budget
    assert srv.deferred > 0
    for r in reqs[:3]:
        alone = ctx.query(torch.from_numpy(r.x).cuda(), sub=-1, what="uvpw").cpu().numpy()
        np.testing.assert_array_equal(r.out, alone)


def test_request_over_budget_is_rejected(server_parts):
    serve, ctx, _, _ = server_parts
    with pytest.raises(ValueError):   # not even one batch slot fits the budget
        serve.QueryServer(ctx, hbm_budget_bytes=1 << 16, n_streams=1, max_batch_points=1 << 16)
    srv = serve.QueryServer(ctx, hbm_budget_bytes=1 << 24, n_streams=1, max_batch_points=1 << 14)
    big = serve.Request(0, 0.0, np.zeros((50000, 3), np.float32))
    with pytest.raises(ValueError):   # larger than a batch slot
        srv.run([big])
