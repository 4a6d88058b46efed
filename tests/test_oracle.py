"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test checks the oracle against mathematics the paper fixes: closed forms,
finite differences, exact Navier-Stokes solutions, invariances of the loss
(section 2.1, 2.2) and the Adam update rule.  A plausible mistake in the
oracle (a dropped term, a wrong sign or index, a transposed operand) fails at
least one of them.
"""
import numpy as np
import pytest

import workloads as wl

TINY_NETS = [(2, 4, 2), (3, 5, 3), (2, 6, 1)]


def rel_err(a, b, floor=None):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    fl = np.sqrt(np.mean(b * b)) if floor is None else floor
    return np.max(np.abs(a - b) / (np.abs(b) + fl + 1e-300))


def rand_theta(dim, W, H, seed, scale=0.7):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(wl.n_params(dim, W, H)) * scale


# ------------------------------------------------------------------ forward
def test_param_count_matches_layout(orc):
    for dim, W, H in [(2, 50, 4), (2, 100, 8), (2, 64, 6), (3, 128, 8)]:
        assert orc.n_params(dim, W, H) == wl.n_params(dim, W, H)
    assert orc.n_params(2, 50, 4) == 8003
    assert orc.n_params(3, 128, 8) == 116740


@pytest.mark.parametrize("dim", [2, 3])
def test_one_hidden_layer_closed_form(orc, dim):
    """H = 1: u_o = sum_k c_ok tanh(w_k . xi + b_k) + e_o, so
    d u_o/d xi_j = sum_k c_ok (1 - s_k^2) w_kj and
    d2 u_o / d x_j^2 = sum_k c_ok (-2 s_k (1 - s_k^2)) w_kj^2."""
    W, D = 7, dim + 1
    rng = np.random.default_rng(3)
    W1 = rng.standard_normal((W, D))
    b1 = rng.standard_normal(W)
    C2 = rng.standard_normal((D, W))
    e = rng.standard_normal(D)
    theta = np.concatenate([W1.ravel(), b1, C2.ravel(), e])
    x = rng.uniform(-1, 1, size=(9, D))
    y = orc.channels(dim, W, 1, theta, x)
    z = x @ W1.T + b1
    s = np.tanh(z)
    s1 = 1 - s * s
    s2 = -2 * s * s1
    np.testing.assert_allclose(y[:, 0, :], s @ C2.T + e, rtol=1e-13, atol=1e-13)
    for j in range(D):            # spatial and time first derivatives
        np.testing.assert_allclose(y[:, 1 + j, :], (s1 * W1[:, j]) @ C2.T, rtol=1e-12, atol=1e-13)
    for j in range(dim):          # spatial second derivatives
        np.testing.assert_allclose(y[:, dim + 2 + j, :], (s2 * W1[:, j] ** 2) @ C2.T,
                                   rtol=1e-12, atol=1e-13)


def test_zero_hidden_weights_give_constant(orc):
    dim, W, H = 2, 6, 3
    th = np.zeros(wl.n_params(dim, W, H))
    th[-3:] = [0.3, -1.2, 2.5]
    x = np.random.default_rng(0).uniform(size=(5, 3))
    y = orc.channels(dim, W, H, th, x)
    assert np.all(y[:, 0, :] == np.array([0.3, -1.2, 2.5]))
    assert np.all(y[:, 1:, :] == 0.0)


@pytest.mark.parametrize("dim,W,H", TINY_NETS)
def test_channels_match_finite_differences(orc, dim, W, H):
    """Derivative channels equal central differences of the value forward."""
    D = dim + 1
    th = rand_theta(dim, W, H, 10 + dim)
    x = np.random.default_rng(1).uniform(-0.8, 0.8, size=(6, D))
    y = orc.channels(dim, W, H, th, x)
    f = lambda pts: orc.values(dim, W, H, th, pts)
    np.testing.assert_allclose(y[:, 0, :], f(x), rtol=0, atol=1e-15)
    h1, h2 = 1e-5, 1e-4
    for j in range(D):
        e = np.zeros(D)
        e[j] = 1.0
        fd1 = (f(x + h1 * e) - f(x - h1 * e)) / (2 * h1)
        assert rel_err(y[:, 1 + j, :], fd1) < 1e-6, j
        if j < dim:
            fd2 = (f(x + h2 * e) - 2 * f(x) + f(x - h2 * e)) / (h2 * h2)
            assert rel_err(y[:, dim + 2 + j, :], fd2) < 1e-5, j


# ---------------------------------------------------------------- residuals
def fd_stack(field, dim, x, h=1e-3):
    """Channel stack of an analytic field by fourth-order central differences."""
    D = dim + 1
    n = x.shape[0]
    C = 2 * dim + 2
    y = np.zeros((n, C, D))
    f = lambda p: np.stack(field(*(p[:, i] for i in range(D))), 1)
    y[:, 0, :] = f(x)
    for j in range(D):
        e = np.zeros(D)
        e[j] = h
        fp2, fp1, fm1, fm2 = f(x + 2 * e), f(x + e), f(x - e), f(x - 2 * e)
        y[:, 1 + j, :] = (-fp2 + 8 * fp1 - 8 * fm1 + fm2) / (12 * h)
        if j < dim:
            y[:, dim + 2 + j, :] = (-fp2 + 16 * fp1 - 30 * y[:, 0, :] + 16 * fm1 - fm2) / (12 * h * h)
    return y


def test_residual_vanishes_taylor_green(orc):
    Re = 100.0
    x = np.random.default_rng(2).uniform(0, 1, size=(50, 3))
    y = fd_stack(lambda a, b, t: wl.taylor_green(a, b, t, Re=Re), 2, x)
    r = orc.residuals(2, 1.0 / Re, y)
    scale = np.abs(y).max()
    assert np.abs(r).max() < 1e-7 * scale
    # every term is active: the convective and pressure terms alone are O(1)
    assert np.abs(y[:, 1 + 0, 2]).max() > 1.0
    # the wrong viscosity leaves a residual
    r_bad = orc.residuals(2, 2.0 / Re, y)
    assert np.abs(r_bad[:, :2]).max() > 1e-2


def test_residual_vanishes_ethier_steinman(orc):
    x = np.random.default_rng(3).uniform(-1, 1, size=(50, 4))
    x[:, 3] = np.abs(x[:, 3])
    y = fd_stack(lambda a, b, c, t: wl.ethier_steinman(a, b, c, t), 3, x)
    r = orc.residuals(3, 1.0, y)
    assert np.abs(r).max() < 1e-7 * np.abs(y).max()
    r_bad = orc.residuals(3, 0.5, y)
    assert np.abs(r_bad[:, :3]).max() > 1e-2


def test_residual_stagnation_flow_exact(orc):
    """u = x, v = -y, p = -(x^2+y^2)/2 is a steady solution for any viscosity;
    with its exact (polynomial) channels the residual is exactly zero."""
    rng = np.random.default_rng(4)
    n = 20
    xs, ys = rng.uniform(-2, 2, n), rng.uniform(-2, 2, n)
    y = np.zeros((n, 6, 3))
    y[:, 0, 0], y[:, 0, 1], y[:, 0, 2] = xs, -ys, -(xs ** 2 + ys ** 2) / 2
    y[:, 1, 0] = 1.0           # u_x
    y[:, 2, 1] = -1.0          # v_y
    y[:, 1, 2] = -xs           # p_x
    y[:, 2, 2] = -ys           # p_y
    r = orc.residuals(2, 0.37, y)
    assert np.all(r == 0.0)
    # a hand-evaluated non-solution: add u_t = 1, u_xx = 2 -> r1 = 1 - nu*2
    y[:, 3, 0] = 1.0
    y[:, 4, 0] = 2.0
    r = orc.residuals(2, 0.37, y)
    np.testing.assert_allclose(r[:, 0], 1.0 - 0.74, rtol=0, atol=1e-15)
    assert np.all(r[:, 1:] == 0.0)


# ------------------------------------------------------------------- losses
def problem_arrays(pb):
    s = pb.subs[0]
    return dict(pde_x=s.pde_x, obs_x=s.obs_x, obs_u=s.obs_u, gh_x=s.gh_x, gh_up=s.gh_up,
                gh_kind=s.gh_kind, anc_x=s.anc_x, anc_p=s.anc_p, is_master=s.is_master)


@pytest.mark.parametrize("dim", [2, 3])
def test_losses_of_constant_network(orc, dim):
    """All hidden weights zero: outputs are the output bias b, every
    derivative vanishes, so r = 0 and each MSE is a plain mean of squared
    differences to b (sum over components, mean over points)."""
    pb = wl.tiny(dim=dim, width=4, depth=2, n_pde=6, n_obs=5, n_gh=6, n_anc=3)
    s = pb.subs[0]
    P = pb.n_params
    th = np.zeros(P)
    b = np.linspace(-0.5, 0.8, dim + 1)
    th[-(dim + 1):] = b
    loss, _ = orc.loss_grad(dim, 4, 2, pb.nu, pb.lam, th, want_grad=False, **problem_arrays(pb))
    obs_u = s.obs_u.astype(np.float64)
    L_obs = np.mean(np.sum((b[:dim] - obs_u) ** 2, 1))
    gt = s.gh_up.astype(np.float64)
    L_ghu = np.mean(np.sum((b[:dim] - gt[:, :dim]) ** 2, 1))
    sp = s.gh_kind == 0
    L_sp = np.sum((b[dim] - gt[sp, dim]) ** 2) / len(gt)
    L_tm = np.sum((b[dim] - gt[~sp, dim]) ** 2) / len(gt)
    L_anc = np.mean((b[dim] - s.anc_p.astype(np.float64)) ** 2)
    expect = [L_obs, 0.0, L_ghu, L_sp, L_tm, L_anc]
    np.testing.assert_allclose(loss[:6], expect, rtol=1e-14, atol=1e-15)
    lam = pb.lam
    np.testing.assert_allclose(loss[6], np.dot(lam, expect), rtol=1e-14)


def test_losses_invariant_to_duplication_and_permutation(orc):
    pb = wl.tiny(dim=2, width=5, depth=2, n_pde=9, n_obs=7, n_gh=6, n_anc=2)
    a = problem_arrays(pb)
    th = pb.subs[0].theta
    L0, g0 = orc.loss_grad(2, 5, 2, pb.nu, pb.lam, th, **a)
    dup = {k: (np.concatenate([v, v]) if isinstance(v, np.ndarray) else v) for k, v in a.items()}
    L1, g1 = orc.loss_grad(2, 5, 2, pb.nu, pb.lam, th, **dup)
    np.testing.assert_allclose(L1, L0, rtol=1e-13)
    np.testing.assert_allclose(g1, g0, rtol=1e-12, atol=1e-15)
    rng = np.random.default_rng(0)
    perm = {}
    for k, v in a.items():
        perm[k] = v
    for grp in [("pde_x",), ("obs_x", "obs_u"), ("gh_x", "gh_up", "gh_kind"), ("anc_x", "anc_p")]:
        idx = rng.permutation(len(a[grp[0]]))
        for k in grp:
            perm[k] = a[k][idx]
    L2, g2 = orc.loss_grad(2, 5, 2, pb.nu, pb.lam, th, **perm)
    np.testing.assert_allclose(L2, L0, rtol=1e-13)
    np.testing.assert_allclose(g2, g0, rtol=1e-11, atol=1e-15)


# ---------------------------------------------------------------- gradients
@pytest.mark.parametrize("dim,W,H", TINY_NETS)
@pytest.mark.parametrize("is_master", [False, True])
def test_gradient_matches_finite_differences(orc, dim, W, H, is_master):
    """Hand-written adjoint vs central differences of the total loss with
    every point set and every weight active."""
    pb = wl.tiny(dim=dim, width=W, depth=H, seed=dim * 10 + H, is_master=is_master)
    a = problem_arrays(pb)
    th = pb.subs[0].theta.astype(np.float64)
    L, g = orc.loss_grad(dim, W, H, pb.nu, pb.lam, th, **a)
    h = 1e-6
    fd = np.zeros_like(th)
    for i in range(th.size):
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd[i] = (orc.loss_grad(dim, W, H, pb.nu, pb.lam, tp, want_grad=False, **a)[0][6]
                 - orc.loss_grad(dim, W, H, pb.nu, pb.lam, tm, want_grad=False, **a)[0][6]) / (2 * h)
    assert rel_err(g, fd) < 1e-6
    assert np.linalg.norm(g - fd) / np.linalg.norm(fd) < 1e-7


def test_gradient_linear_in_weights(orc):
    """grad L(lambda) = sum_i lambda_i grad L_i, with each L_i isolated by a
    one-hot weight vector; the one-hot totals equal the unweighted terms."""
    pb = wl.tiny(dim=3, width=4, depth=2)
    a = problem_arrays(pb)
    th = pb.subs[0].theta
    L, g = orc.loss_grad(3, 4, 2, pb.nu, pb.lam, th, **a)
    acc = np.zeros_like(g)
    for i in range(6):
        e = np.zeros(6)
        e[i] = 1.0
        Li, gi = orc.loss_grad(3, 4, 2, pb.nu, e, th, **a)
        assert Li[6] == pytest.approx(L[i], rel=1e-14)
        acc += pb.lam[i] * gi
    np.testing.assert_allclose(acc, g, rtol=1e-10, atol=1e-14)


def test_hidden_unit_permutation_permutes_gradient(orc):
    dim, W, H = 2, 5, 2
    pb = wl.tiny(dim=dim, width=W, depth=H)
    a = problem_arrays(pb)
    th = pb.subs[0].theta.astype(np.float64)
    D = dim + 1
    perm = np.array([3, 0, 4, 1, 2])

    def unpack(t):
        o = 0
        parts = []
        for fo, fi in [(W, D), (W, W), (D, W)]:
            Wm = t[o:o + fo * fi].reshape(fo, fi); o += fo * fi
            b = t[o:o + fo]; o += fo
            parts.append((Wm, b))
        return parts

    def pack(parts):
        return np.concatenate([np.concatenate([Wm.ravel(), b]) for Wm, b in parts])

    def permute(t):
        (W1, b1), (W2, b2), (W3, b3) = unpack(t)
        # permute units of hidden layer 1
        return pack([(W1[perm], b1[perm]), (W2[:, perm], b2), (W3, b3)])

    L0, g0 = orc.loss_grad(dim, W, H, pb.nu, pb.lam, th, **a)
    L1, g1 = orc.loss_grad(dim, W, H, pb.nu, pb.lam, permute(th), **a)
    assert L1[6] == pytest.approx(L0[6], rel=1e-13)
    np.testing.assert_allclose(g1, permute(g0), rtol=1e-11, atol=1e-15)


def test_pressure_gauge_invariance(orc):
    """p enters the Navier-Stokes residuals only through grad p (section 2.2):
    shifting the pressure output bias leaves L_PDE and L_obs unchanged and
    their derivative with respect to that bias is zero; the anchor and ghost
    pressure terms change by the stated amounts."""
    dim, W, H = 2, 5, 3
    pb = wl.tiny(dim=dim, width=W, depth=H)
    a = problem_arrays(pb)
    th = pb.subs[0].theta.astype(np.float64)
    c = 0.37
    ts = th.copy()
    ts[-1] += c
    L0, g0 = orc.loss_grad(dim, W, H, pb.nu, pb.lam, th, **a)
    L1, _ = orc.loss_grad(dim, W, H, pb.nu, pb.lam, ts, **a)
    assert abs(L1[1] - L0[1]) <= 1e-14 * max(1.0, L0[1])
    assert L1[0] == L0[0]
    lam_phys = np.array([1.0, 1.0, 0.0, 0.0, 0.0, 0.0])
    _, gp = orc.loss_grad(dim, W, H, pb.nu, lam_phys, th, **a)
    assert abs(gp[-1]) < 1e-14
    # the anchor term changes by exactly the shift of its squared errors
    s = pb.subs[0]
    p_anc = orc.values(dim, W, H, th, s.anc_x)[:, dim]
    dL = np.mean((p_anc + c - s.anc_p) ** 2 - (p_anc - s.anc_p) ** 2)
    assert L1[5] - L0[5] == pytest.approx(dL, rel=1e-10)


def test_master_ignores_spatial_ghost_pressure(orc):
    pb = wl.tiny(dim=2, width=4, depth=2)
    a = problem_arrays(pb)
    th = pb.subs[0].theta
    a_m = dict(a, is_master=True)
    Lm, gm = orc.loss_grad(2, 4, 2, pb.nu, pb.lam, th, **a_m)
    lam0 = pb.lam.copy()
    lam0[3] = 0.0
    Ls, gs = orc.loss_grad(2, 4, 2, pb.nu, lam0, th, **dict(a, is_master=False))
    np.testing.assert_allclose(gm, gs, rtol=0, atol=0)
    assert Lm[6] == Ls[6]
    assert Lm[3] > 0  # the term itself is still reported


# --------------------------------------------------------------------- adam
def test_adam_first_step_closed_form(orc):
    rng = np.random.default_rng(5)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50) * 10.0 ** rng.uniform(-6, 1, 50)
    t1, m1, v1 = orc.adam(th, np.zeros(50), np.zeros(50), g, 1, lr=1e-3)
    np.testing.assert_allclose(t1, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-14)
    # second step, values by hand
    g2 = np.full(50, 2.0)
    t2, m2, v2 = orc.adam(t1, m1, v1, g2, 2, lr=1e-3)
    m_hand = 0.9 * 0.1 * g + 0.1 * 2.0
    v_hand = 0.999 * 0.001 * g * g + 0.001 * 4.0
    step = 1e-3 * (m_hand / (1 - 0.81)) / (np.sqrt(v_hand / (1 - 0.999 ** 2)) + 1e-8)
    np.testing.assert_allclose(t2, t1 - step, rtol=1e-13)


# ------------------------------------------------------------ routing/query
def test_route_half_open_boxes(orc):
    boxes = wl.strip_geometry(4, 4)
    pts = np.array([[0.0, 0.0, 0.0],      # corner -> 0
                    [2.0, 1.0, 0.5],      # on x = 2 face -> strip 1
                    [8.0, 2.0, 4.0],      # global upper corner -> last
                    [1.0, 1.0, 1.0],      # t = 1 face -> slab 1
                    [8.5, 1.0, 1.0],      # outside
                    [7.99, 1.99, 3.99]])
    sub = orc.route(2, boxes, pts)
    assert list(sub) == [0, 1, 15, 4, -1, 15]


def test_query_equals_channels(orc):
    boxes, thetas = wl.serving_nets(seed=0, width=6, depth=2)
    rng = np.random.default_rng(6)
    x = wl.query_points(rng, 40).astype(np.float64)
    out = orc.query2d(6, 2, thetas, boxes, x)
    sub = orc.route(2, boxes, x)
    for i in range(len(x)):
        y = orc.channels(2, 6, 2, thetas[sub[i]], x[i:i + 1])[0]
        assert out[i, 0] == y[0, 0] and out[i, 1] == y[0, 1] and out[i, 2] == y[0, 2]
        assert out[i, 3] == y[1, 1] - y[2, 0]


def test_exchange_anchor_normalisation(orc):
    dim, W, H = 2, 5, 2
    th = rand_theta(dim, W, H, 7)
    x_anc = np.array([1.0, 1.0])
    ts = np.linspace(0, 1, 7)
    x = np.stack([np.full(7, 1.0), np.full(7, 1.0), ts], 1)
    out = orc.exchange(dim, W, H, th, True, x_anc, x)
    assert np.all(out[:, dim] == 0.0)
    raw = orc.values(dim, W, H, th, x)
    np.testing.assert_array_equal(out[:, :dim], raw[:, :dim])
    # non-master senders pass raw pressure
    out2 = orc.exchange(dim, W, H, th, False, x_anc, x)
    np.testing.assert_array_equal(out2, raw)
    # elsewhere the master's target is p(x,t) - p(x_anc,t)
    y = np.array([[0.3, 0.2, 0.6]])
    o = orc.exchange(dim, W, H, th, True, x_anc, y)
    pa = orc.values(dim, W, H, th, np.array([[1.0, 1.0, 0.6]]))[0, dim]
    assert o[0, dim] == pytest.approx(orc.values(dim, W, H, th, y)[0, dim] - pa, abs=1e-15)


def test_oracle_thread_count_does_not_change_results(orc):
    pb = wl.config1(0)
    s = pb.subs[0]
    a = problem_arrays(pb)
    orc.threads(1)
    L1, g1 = orc.loss_grad(2, 50, 4, pb.nu, pb.lam, s.theta, **a)
    orc.threads(4)
    L4, g4 = orc.loss_grad(2, 50, 4, pb.nu, pb.lam, s.theta, **a)
    orc.threads(0)
    np.testing.assert_allclose(L4, L1, rtol=1e-13)
    np.testing.assert_allclose(g4, g1, rtol=1e-10, atol=1e-16)


@pytest.mark.parametrize("dim", [2, 3])
def test_pde_loss_is_mean_of_squared_residuals(orc, dim):
    """L_PDE of a generic network equals (1/N) sum_n sum_k r_k^2 built from the
    separately pinned channel stack and residual entry points."""
    pb = wl.tiny(dim=dim, width=6, depth=2, n_pde=11)
    s = pb.subs[0]
    L, _ = orc.loss_grad(dim, 6, 2, pb.nu, pb.lam, s.theta, want_grad=False, **problem_arrays(pb))
    r = orc.residuals(dim, pb.nu, orc.channels(dim, 6, 2, s.theta, s.pde_x))
    assert L[1] == pytest.approx(np.mean(np.sum(r * r, 1)), rel=1e-13)
    assert L[1] > 1e-3


# ------------------------------------------- sine activation, 3D recipe
@pytest.fixture
def sin_act(orc):
    orc.set_activation("sin")
    yield orc
    orc.set_activation("tanh")


@pytest.mark.parametrize("dim", [2, 3])
def test_sine_one_hidden_layer_closed_form(sin_act, dim):
    """H = 1 with sin: u = sum c sin(w.xi + b) + e, u_j = sum c cos(.) w_j,
    u_jj = -sum c sin(.) w_j^2."""
    orc = sin_act
    W, D = 6, dim + 1
    rng = np.random.default_rng(8)
    W1, b1 = rng.standard_normal((W, D)), rng.standard_normal(W)
    C2, e = rng.standard_normal((D, W)), rng.standard_normal(D)
    theta = np.concatenate([W1.ravel(), b1, C2.ravel(), e])
    x = rng.uniform(-1, 1, size=(7, D))
    y = orc.channels(dim, W, 1, theta, x)
    z = x @ W1.T + b1
    np.testing.assert_allclose(y[:, 0, :], np.sin(z) @ C2.T + e, rtol=1e-13, atol=1e-13)
    for j in range(D):
        np.testing.assert_allclose(y[:, 1 + j, :], (np.cos(z) * W1[:, j]) @ C2.T, rtol=1e-12, atol=1e-13)
    for j in range(dim):
        np.testing.assert_allclose(y[:, dim + 2 + j, :], (-np.sin(z) * W1[:, j] ** 2) @ C2.T,
                                   rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("dim,W,H", TINY_NETS[:2])
def test_sine_channels_and_gradient_match_finite_differences(sin_act, dim, W, H):
    orc = sin_act
    D = dim + 1
    th = rand_theta(dim, W, H, 20 + dim)
    x = np.random.default_rng(2).uniform(-0.8, 0.8, size=(5, D))
    y = orc.channels(dim, W, H, th, x)
    f = lambda pts: orc.values(dim, W, H, th, pts)
    for j in range(D):
        e = np.zeros(D)
        e[j] = 1.0
        fd1 = (f(x + 1e-5 * e) - f(x - 1e-5 * e)) / 2e-5
        assert rel_err(y[:, 1 + j, :], fd1) < 1e-6
        if j < dim:
            fd2 = (f(x + 1e-4 * e) - 2 * f(x) + f(x - 1e-4 * e)) / 1e-8
            assert rel_err(y[:, dim + 2 + j, :], fd2) < 1e-5
    pb = wl.tiny(dim=dim, width=W, depth=H, seed=31)
    a = problem_arrays(pb)
    t0 = pb.subs[0].theta.astype(np.float64)
    _, g = orc.loss_grad(dim, W, H, pb.nu, pb.lam, t0, **a)
    fd = np.zeros_like(t0)
    for i in range(t0.size):
        tp, tm = t0.copy(), t0.copy()
        tp[i] += 1e-6
        tm[i] -= 1e-6
        fd[i] = (orc.loss_grad(dim, W, H, pb.nu, pb.lam, tp, want_grad=False, **a)[0][6]
                 - orc.loss_grad(dim, W, H, pb.nu, pb.lam, tm, want_grad=False, **a)[0][6]) / 2e-6
    assert rel_err(g, fd) < 1e-6


def test_component_weights_by_hand(orc):
    """Weighted velocity components in L_obs and L_gh_u (section 3.3): with a
    constant network each term is a plain weighted mean of squares."""
    dim = 3
    pb = wl.tiny(dim=dim, width=4, depth=2, n_pde=3, n_obs=6, n_gh=5, n_anc=0)
    s = pb.subs[0]
    th = np.zeros(pb.n_params)
    b = np.array([0.2, -0.4, 0.7, 0.1])
    th[-4:] = b
    w = np.array([1.0, 5.0, 100.0])
    orc.set_component_weights(w)
    try:
        L, g = orc.loss_grad(dim, 4, 2, pb.nu, pb.lam, th, **problem_arrays(pb))
        La, ga = orc.loss_grad(dim, 4, 2, pb.nu, pb.lam, th + 0.01, **problem_arrays(pb))
    finally:
        orc.set_component_weights(None)
    L_obs = np.mean(np.sum(w * (b[:3] - s.obs_u.astype(np.float64)) ** 2, 1))
    L_ghu = np.mean(np.sum(w * (b[:3] - s.gh_up[:, :3].astype(np.float64)) ** 2, 1))
    assert L[0] == pytest.approx(L_obs, rel=1e-13)
    assert L[2] == pytest.approx(L_ghu, rel=1e-13)
    # the pressure terms are untouched by the velocity weights
    L1, _ = orc.loss_grad(dim, 4, 2, pb.nu, pb.lam, th, **problem_arrays(pb))
    np.testing.assert_array_equal(L[3:6], L1[3:6])
    # and the weighted gradient still matches finite differences
    orc.set_component_weights(w)
    try:
        pbt = wl.tiny(dim=3, width=4, depth=2, seed=5)
        a = problem_arrays(pbt)
        t0 = pbt.subs[0].theta.astype(np.float64)
        _, g = orc.loss_grad(3, 4, 2, pbt.nu, pbt.lam, t0, **a)
        i = np.argmax(np.abs(g))
        tp, tm = t0.copy(), t0.copy()
        tp[i] += 1e-6
        tm[i] -= 1e-6
        fd = (orc.loss_grad(3, 4, 2, pbt.nu, pbt.lam, tp, want_grad=False, **a)[0][6]
              - orc.loss_grad(3, 4, 2, pbt.nu, pbt.lam, tm, want_grad=False, **a)[0][6]) / 2e-6
        assert fd == pytest.approx(g[i], rel=1e-6)
    finally:
        orc.set_component_weights(None)


def test_gradient_clipping_closed_form(orc):
    g = np.array([3.0, 4.0, 0.0, -12.0])          # norm 13
    c, n = orc.clip_grad(g, 1.0)
    assert n == 13.0
    np.testing.assert_allclose(c, g / 13.0, rtol=1e-15)
    assert np.linalg.norm(c) == pytest.approx(1.0, rel=1e-15)
    c2, _ = orc.clip_grad(g, 20.0)                 # below the limit: unchanged
    np.testing.assert_array_equal(c2, g)
    c3, _ = orc.clip_grad(g, 0.0)                  # 0 disables clipping
    np.testing.assert_array_equal(c3, g)


def test_step_lr_schedule_by_hand(orc):
    # appendix B 3D cylinder: factor 0.3 every 5k epochs
    assert orc.step_lr(1e-3, 0.3, 5000, 1) == 1e-3
    assert orc.step_lr(1e-3, 0.3, 5000, 5000) == 1e-3
    assert orc.step_lr(1e-3, 0.3, 5000, 5001) == pytest.approx(3e-4, rel=1e-15)
    assert orc.step_lr(1e-3, 0.3, 5000, 10001) == pytest.approx(9e-5, rel=1e-15)
    assert orc.step_lr(1e-3, 0.3, 0, 10001) == 1e-3


# ------------------------------------------------ evaluation post-processing
def _eval_setup(orc, masters=(0, 4, 8, 12)):
    boxes, thetas = wl.serving_nets(seed=4, width=6, depth=2)
    is_master = [s in masters for s in range(len(thetas))]
    rng = np.random.default_rng(12)
    # 3 snapshots on a uniform spatial grid at t = 0.25, 1.5, 2.75
    gx, gy = np.meshgrid(np.linspace(0.05, 7.95, 20), np.linspace(0.05, 1.95, 8))
    pts, off = [], [0]
    for t in (0.25, 1.5, 2.75):
        pts.append(np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, t)], 1))
        off.append(off[-1] + gx.size)
    x = np.concatenate(pts)
    return boxes, thetas, is_master, x, np.array(off), rng


def test_evaluation_identity_gives_zero_error(orc):
    """Reference = the stitched raw network output: velocity errors vanish, and
    with every subdomain of a snapshot a master the anchor offset is constant
    per snapshot, so mean removal cancels it and the pressure error vanishes."""
    boxes, thetas, _, x, off, _ = _eval_setup(orc)
    every = [True] * len(thetas)
    sub = orc.route(2, boxes, x)
    ref = np.array([orc.values(2, 6, 2, thetas[s], x[i:i + 1])[0] for i, s in enumerate(sub)])
    # one master subdomain per snapshot region: restrict x to the first strip
    keep = (x[:, 0] < 2.0)
    xs, rs = x[keep], ref[keep]
    offs = np.concatenate([[0], np.cumsum([np.sum(keep[off[k]:off[k + 1]]) for k in range(3)])])
    err = orc.evaluate(2, 6, 2, thetas, every, boxes, [1.0, 1.0], xs, rs, offs)
    assert np.all(err[:3] == 0.0)
    assert err[3] < 1e-13


def test_evaluation_closed_forms(orc):
    boxes, thetas, is_master, x, off, rng = _eval_setup(orc)
    sub = orc.route(2, boxes, x)
    raw = np.array([orc.values(2, 6, 2, thetas[s], x[i:i + 1])[0] for i, s in enumerate(sub)])
    # processed prediction by hand: anchor subtraction on masters
    pred = raw.copy()
    for i, s in enumerate(sub):
        if is_master[s]:
            pred[i, 2] -= orc.values(2, 6, 2, thetas[s], np.array([[1.0, 1.0, x[i, 2]]]))[0, 2]
    # reference = 2 x processed prediction: every relative error is 1/2
    ref = 2.0 * pred
    err = orc.evaluate(2, 6, 2, thetas, is_master, boxes, [1.0, 1.0], x, ref, off)
    np.testing.assert_allclose(err, 0.5, rtol=1e-12)
    # a per-snapshot constant added to the reference pressure changes nothing
    ref2 = ref.copy()
    for k, c in enumerate([3.0, -7.0, 0.5]):
        ref2[off[k]:off[k + 1], 2] += c
    err2 = orc.evaluate(2, 6, 2, thetas, is_master, boxes, [1.0, 1.0], x, ref2, off)
    np.testing.assert_allclose(err2, err, rtol=1e-12)
    # but a non-constant pressure change does
    ref3 = ref.copy()
    ref3[:, 2] += x[:, 0]
    err3 = orc.evaluate(2, 6, 2, thetas, is_master, boxes, [1.0, 1.0], x, ref3, off)
    assert abs(err3[3] - err[3]) > 1e-3
    np.testing.assert_array_equal(err3[:3], err[:3])
