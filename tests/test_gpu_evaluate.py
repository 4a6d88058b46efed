"""Evaluation post-processing on the GPU (section 3: stitched prediction,
master anchor pinning, per-snapshot pressure-mean removal, relative L2)
against the FP64 oracle."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# The errors are ratios of sums of squares accumulated in float32 over a few
# thousand points (blockwise, then across blocks): relative rounding of such a
# sum is a few 1e-7 times the number of summation levels, far below 1e-4.
EVAL_RTOL = 1e-4


def _snapshots(rng, sizes, lo, hi):
    """Points of each snapshot at one time t_k (uniform in space), in order."""
    xs, off = [], [0]
    dim = len(lo) - 1
    for k, n in enumerate(sizes):
        t = lo[-1] + (hi[-1] - lo[-1]) * (k + 0.5) / len(sizes)
        p = wl.uniform(rng, n, lo[:dim], hi[:dim])
        xs.append(np.concatenate([p, np.full((n, 1), t, np.float32)], axis=1))
        off.append(off[-1] + n)
    return np.concatenate(xs).astype(np.float32), np.asarray(off, np.int64)


def _run(serve, boxes, thetas, masters, width, depth, dim, act, x, ref, off, x_anc, orc):
    ctx = serve.serving_context(boxes, thetas, width, depth, dim=dim, device="cuda",
                                masters=masters, activation=act)
    try:
        err = ctx.evaluate(torch.from_numpy(x).cuda(), torch.from_numpy(ref).cuda(), off, x_anc)
        got = err.cpu().numpy().astype(np.float64)
    finally:
        ctx.close()
    orc.set_activation(act)
    try:
        want = orc.evaluate(dim, width, depth, thetas, masters, boxes, x_anc, x.astype(np.float64),
                            ref.astype(np.float64), off)
    finally:
        orc.set_activation("tanh")
    return got, want


@pytest.fixture(scope="module")
def serve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_15883_amd import serve as s
    return s


def test_evaluate_2d_strips_matches_oracle(serve, orc):
    """16 tanh networks on 4 strips x 4 time slabs, masters = first strip;
    ragged snapshots (one of a single point, one empty, several spanning more
    than one reduction block)."""
    boxes, thetas = wl.serving_nets(seed=3, width=24, depth=3)
    masters = [s % 4 == 0 for s in range(16)]
    rng = np.random.default_rng(11)
    x, off = _snapshots(rng, [3000, 1, 0, 2500, 1025, 777], (0, 0, 0), (8, 2, 4))
    u, v, p = wl.taylor_green(x[:, 0].astype(np.float64), x[:, 1], x[:, 2])
    ref = np.stack([u, v, p], axis=1).astype(np.float32)
    got, want = _run(serve, boxes, thetas, masters, 24, 3, 2, "tanh", x, ref, off, [1.0, 1.0], orc)
    assert np.all(np.isfinite(want))
    np.testing.assert_allclose(got, want, rtol=EVAL_RTOL)


def test_evaluate_reference_equal_to_prediction(serve, orc):
    """Reference = the processed prediction (computed here from oracle network
    values) plus a per-snapshot constant in pressure: every error is (close
    to) zero."""
    boxes, thetas = wl.serving_nets(seed=5, width=16, depth=2)
    masters = [s % 4 == 0 for s in range(16)]
    rng = np.random.default_rng(12)
    x, off = _snapshots(rng, [1500, 2048, 999], (0, 0, 0), (8, 2, 4))
    # processed prediction from the oracle (master anchor subtraction)
    sub = orc.route(2, boxes, x.astype(np.float64))
    pred = np.zeros((x.shape[0], 3))
    for s in range(16):
        idx = np.nonzero(sub == s)[0]
        if idx.size == 0:
            continue
        pred[idx] = orc.values(2, 16, 2, thetas[s], x[idx].astype(np.float64))
        if masters[s]:
            xa = np.concatenate([np.ones((idx.size, 2)), x[idx, 2:3].astype(np.float64)], axis=1)
            pred[idx, 2] -= orc.values(2, 16, 2, thetas[s], xa)[:, 2]
    for k in range(3):
        pred[off[k]:off[k + 1], 2] += 10.0 * (k + 1)
    ref = pred.astype(np.float32)
    got, want = _run(serve, boxes, thetas, masters, 16, 2, 2, "tanh", x, ref, off, [1.0, 1.0], orc)
    # the reference is rounded to float32 (pressure offsets up to 30): the
    # oracle's own errors are of the order of float32 epsilon times 30 / spread
    assert np.all(want < 1e-5)
    assert np.all(got < 1e-4)


def test_evaluate_3d_sine_matches_oracle(serve, orc):
    """Two 3D sine networks split along x, the master holding the anchor."""
    width, depth = 32, 3
    boxes = np.array([[[0, 0, 0, 0], [1, 1, 1, 1]], [[1, 0, 0, 0], [2, 1, 1, 1]]], np.float64)
    thetas = [wl.xavier_theta(3, width, depth, 40 + s) for s in range(2)]
    masters = [True, False]
    rng = np.random.default_rng(13)
    x, off = _snapshots(rng, [2100, 700, 1], (0, 0, 0, 0), (2, 1, 1, 1))
    u, v, w, p = wl.ethier_steinman(*(x[:, q].astype(np.float64) for q in range(4)))
    ref = np.stack([u, v, w, p], axis=1).astype(np.float32)
    got, want = _run(serve, boxes, thetas, masters, width, depth, 3, "sin", x, ref, off,
                     [0.5, 0.5, 0.5], orc)
    np.testing.assert_allclose(got, want, rtol=EVAL_RTOL)


def test_evaluate_rejects_bad_snapshots(serve):
    boxes, thetas = wl.serving_nets(seed=3, width=16, depth=2)
    ctx = serve.serving_context(boxes, thetas, 16, 2, device="cuda")
    try:
        x = torch.zeros(10, 3, device="cuda")
        from paper_2602_15883_amd.abi import PinnError
        with pytest.raises(PinnError):
            ctx.evaluate(x, x, [0, 4], [1.0, 1.0])          # does not end at n
        with pytest.raises(PinnError):
            ctx.evaluate(x, x, [0, 6, 4, 10], [1.0, 1.0])   # decreasing
    finally:
        ctx.close()
