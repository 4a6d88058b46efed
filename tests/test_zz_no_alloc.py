"""pinn_query_noalloc: the routed query on the library-held device scratch
(for callers that cannot allocate).  Through the C ABI, against pinn_query
with caller scratch (the same kernels: bitwise equal) and the oracle, on two
calls in a row (the second smaller, over the stale contents of the first),
from two contexts on the same GPU, and the size limit."""
import ctypes

import numpy as np
import pytest

import workloads as wl
from parity import assert_close

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

LIMIT = 1 << 20


@pytest.fixture(scope="module")
def parts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_15883_amd import abi
    from paper_2602_15883_amd.serve import serving_context
    boxes, thetas = wl.serving_nets(seed=5, width=40, depth=3)
    ctx = serving_context(boxes, thetas, 40, 3, device="cuda", max_query_points=1 << 22)
    yield abi, ctx, boxes, thetas
    ctx.close()


def _noalloc(abi, ctx, x, out, sub=-1, what=1):
    st = abi.lib().pinn_query_noalloc(ctx._h, ctypes.c_void_p(x.data_ptr()), x.shape[0], sub, what,
                                      ctypes.c_void_p(out.data_ptr()), None)
    return st


def _with_scratch(abi, ctx, x, sub=-1, what=1):
    n = x.shape[0]
    cols = 4 if what == 1 else 3
    out = torch.empty(n, cols, dtype=torch.float32, device="cuda")
    need = int(abi.lib().pinn_query_scratch_bytes(ctx._h, n))
    scratch = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    base = scratch.data_ptr() + (-scratch.data_ptr()) % 256
    st = abi.lib().pinn_query(ctx._h, ctypes.c_void_p(x.data_ptr()), n, sub, what,
                              ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(base), need, None)
    assert st == abi.PINN_OK
    return out


def test_two_calls_second_smaller(parts, orc):
    abi, ctx, boxes, thetas = parts
    rng = np.random.default_rng(12)
    for n in (30_001, 5_000):            # multi-block routing, then the one-workgroup path
        x = wl.query_points(rng, n)
        x[0] = [8.0, 2.0, 4.0]           # the global upper corner
        x[1] = [2.0, 1.0, 1.0]           # on the faces of four boxes
        xt = torch.from_numpy(x).cuda()
        out = torch.full((n, 4), -7.0, dtype=torch.float32, device="cuda")
        print(f"pinn_query_noalloc routed uvpw n={n}", flush=True)
        assert _noalloc(abi, ctx, xt, out) == abi.PINN_OK
        ref = _with_scratch(abi, ctx, xt)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        np.testing.assert_array_equal(got, ref.cpu().numpy())
        orc_ref = orc.query2d(40, 3, thetas, boxes, x[:3000])
        assert_close(got[:3000, :3], orc_ref[:, :3], 1e-5, "uvp")
        assert_close(got[:3000, 3], orc_ref[:, 3], 1e-4, "vorticity")


def test_single_subdomain_and_second_context(parts):
    abi, ctx, boxes, thetas = parts
    from paper_2602_15883_amd.serve import serving_context
    x = torch.from_numpy(wl.query_points(np.random.default_rng(13), 20_000)).cuda()
    out = torch.empty(20_000, 3, dtype=torch.float32, device="cuda")
    assert _noalloc(abi, ctx, x, out, sub=3, what=0) == abi.PINN_OK
    ref = _with_scratch(abi, ctx, x, sub=3, what=0)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), ref.cpu().numpy())
    # a second context on the same GPU shares the array: calls in order agree
    ctx2 = serving_context(boxes, thetas[::-1], 40, 3, device="cuda")
    try:
        for c in (ctx2, ctx, ctx2):
            o = torch.empty(20_000, 4, dtype=torch.float32, device="cuda")
            assert _noalloc(abi, c, x, o) == abi.PINN_OK
            r = _with_scratch(abi, c, x)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(o.cpu().numpy(), r.cpu().numpy())
    finally:
        ctx2.close()


def test_limit_rejected_before_launch(parts):
    abi, ctx, _, _ = parts
    n = LIMIT + 1
    x = torch.zeros(n, 3, dtype=torch.float32, device="cuda")
    out = torch.full((n, 4), 5.0, dtype=torch.float32, device="cuda")
    assert _noalloc(abi, ctx, x, out) == abi.PINN_E_BUDGET
    assert b"library-held scratch" in abi.lib().pinn_last_error()
    torch.cuda.synchronize()
    assert bool((out == 5.0).all())
