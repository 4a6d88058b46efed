"""Memory check of the workspace layout: with pinn_config.guard_bytes > 0 every
region of the caller's workspace (items, ranges, counters, slabs, stash,
partial sums, weight fragments, loss, gradient, clip, boxes, exchange items,
targets) is followed by a guard zone that pinn_create fills with a pattern.
After steps in every launch mode, routed queries and an exchange, no zone may
have lost a byte of its pattern: no kernel wrote outside its region.  The
shapes cover the one-row-block kernel (7 and 8 waves), the two-stack plan with
the K-split of two extra row blocks and several tiles per workgroup, the
column-split plan, and grouped subdomains with 2 workgroups per compute unit."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GUARD = 4096


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_15883_amd as P
    P.lib()
    return P


def _exercise(ctx, pb):
    ctx.step(1, update=False, want_grad=True)
    ctx.step(2)
    ctx.step(3, time_kernel=True)
    ctx.kernel_time()
    ctx.step(4, update=False, want_grad=True, per_subdomain=True)
    x = torch.from_numpy(np.ascontiguousarray(pb.subs[0].pde_x[:500], dtype=np.float32)).cuda()
    ctx.query(x, sub=0, what="channels")
    if len(pb.subs) > 1 and pb.dim == 2:
        xq = wl.query_points(np.random.default_rng(3), 3000)
        ctx.query(torch.from_numpy(np.ascontiguousarray(xq, dtype=np.float32)).cuda(), sub=-1, what="uvpw")
    torch.cuda.synchronize()


@pytest.mark.parametrize("dim,W,H,act,npde", [
    (3, 128, 3, "tanh", 5000),    # one row block per wave, 8 waves
    (2, 100, 3, "sin", 5000),     # 7 waves (W padded to 112)
    (2, 150, 2, "tanh", 8201),    # two-stack plan with the K-split, several tiles per workgroup
    (3, 200, 2, "sin", 3000),     # column-split plan
])
def test_single_subdomain_writes_stay_in_their_regions(pkg, dim, W, H, act, npde):
    pb = wl.tiny(dim=dim, width=W, depth=H, n_pde=npde, n_obs=150, n_gh=30, n_anc=2, seed=W + H)
    pb.activation = act
    print(f"guards dim={dim} W={W} H={H} act={act} n_pde={npde}", flush=True)
    ctx = pkg.context_from_problem(pb, device="cuda", graph=True, guard_bytes=GUARD)
    try:
        assert ctx.check_guards() == 0
        _exercise(ctx, pb)
        assert ctx.check_guards() == 0
    finally:
        ctx.close()


def test_grouped_with_exchange_writes_stay_in_their_regions(pkg):
    pb = wl.config3(0, width=64, depth=3, pde_range=(100, 900), n_obs=20, n_gh_face=40)
    print("guards grouped", flush=True)
    ctx = pkg.context_from_problem(pb, device="cuda", graph=True, guard_bytes=GUARD, blocks_per_cu=2)
    try:
        faces, targets = [], []
        for a, s in enumerate(pb.subs):
            for (b, kind, first, count) in s.faces:
                faces.append((a, b, first, count))
            targets.append(torch.zeros(s.gh_x.shape[0], 3, dtype=torch.float32, device="cuda"))
        ctx.exchange(faces, pb.x_anc, targets)
        _exercise(ctx, pb)
        ctx.exchange(faces[: len(faces) // 2], pb.x_anc, targets)
        torch.cuda.synchronize()
        assert ctx.check_guards() == 0
    finally:
        ctx.close()


def test_guard_check_sees_a_host_write_and_rejects_bad_sizes(pkg):
    """Positive control: clearing the whole workspace from the host clears
    every guard zone, and the check counts all of their bytes; sizes that are
    not a multiple of 256 or exceed 1 MiB are refused."""
    pb = wl.tiny(dim=2, width=20, depth=2, n_pde=40, seed=1)
    ctx = pkg.context_from_problem(pb, device="cuda", graph=False, guard_bytes=512)
    try:
        assert ctx.check_guards() == 0
        ctx.workspace.zero_()
        torch.cuda.synchronize()
        bad = ctx.check_guards()
        assert bad > 0 and bad % 512 == 0
    finally:
        ctx.close()
    ctx = pkg.context_from_problem(pb, device="cuda", graph=False)
    try:
        assert ctx.check_guards() == 0
    finally:
        ctx.close()
    for gb in (100, 2 << 20, -256):
        with pytest.raises(pkg.PinnError):
            pkg.context_from_problem(pb, device="cuda", guard_bytes=gb)


def test_routed_query_stays_in_its_scratch_and_output(pkg):
    """The caller's query scratch and output buffers: a routed query of n
    points writes only the first pinn_query_scratch_bytes(n) bytes of the
    scratch and the first n rows of the output (tails filled with a pattern
    stay intact), for sizes on both sides of the one-workgroup routing path."""
    boxes, thetas = wl.serving_nets(seed=4, width=100, depth=3)
    subs = [wl._sub(2, boxes[s][0], boxes[s][1], thetas[s]) for s in range(len(thetas))]
    pb = wl.Problem("serve_guard", 2, 100, 3, 0.01, np.ones(6), 1e-3, subs)
    ctx = pkg.context_from_problem(pb, device="cuda", graph=False)
    try:
        rng = np.random.default_rng(8)
        for n in (1, 700, 8192, 8193, 50000):
            x = torch.from_numpy(np.ascontiguousarray(wl.query_points(rng, n), dtype=np.float32)).cuda()
            need = ctx.query_scratch_bytes(n)
            scratch = torch.full((need + 256 + GUARD,), 0xA5, dtype=torch.uint8, device="cuda")
            off = (-scratch.data_ptr()) % 256
            used = off + need
            out = torch.full((n + 64, 4), -7.0, dtype=torch.float32, device="cuda")
            # the binding passes the whole tensor; the library must keep to `need`
            ctx.query(x, sub=-1, what="uvpw", out=out[:n], scratch=scratch)
            torch.cuda.synchronize()
            assert int((scratch[used:] != 0xA5).sum()) == 0, f"scratch tail written, n={n}"
            assert bool((out[n:] == -7.0).all()), f"output rows past n written, n={n}"
    finally:
        ctx.close()


def test_exchange_writes_only_the_rows_of_its_faces(pkg):
    """Ghost targets of the faces not exchanged, and the rows around each
    exchanged face, keep their sentinel value."""
    pb = wl.config3(2, width=64, depth=2, pde_range=(50, 100), n_obs=10, n_gh_face=30)
    ctx = pkg.context_from_problem(pb, device="cuda", graph=False)
    try:
        faces = [(a, b, first, count) for a, s in enumerate(pb.subs) for (b, kind, first, count) in s.faces]
        chosen = faces[::2]
        targets = [torch.full((s.gh_x.shape[0], 3), 123.0, dtype=torch.float32, device="cuda")
                   for s in pb.subs]
        ctx.exchange(chosen, pb.x_anc, targets)
        torch.cuda.synchronize()
        for a, s in enumerate(pb.subs):
            mask = np.zeros(s.gh_x.shape[0], dtype=bool)
            for (fa, b, first, count) in chosen:
                if fa == a:
                    mask[first:first + count] = True
            t = targets[a].cpu().numpy()
            assert np.all(t[~mask] == 123.0), f"sub {a}: rows outside its exchanged faces written"
            if mask.any():
                assert np.all(t[mask] != 123.0), f"sub {a}: rows of an exchanged face left unwritten"
    finally:
        ctx.close()
