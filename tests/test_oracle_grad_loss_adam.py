"""Pins of the oracle's loss, parameter gradient, Adam step and schedule scalars:
scipy's Gaussian filter, SSIM(x, x) = 1, central finite differences in FP64,
torch.optim.Adam in FP64, and closed forms of Eq. 3-8."""
import math

import numpy as np
import pytest
import torch
from scipy.ndimage import gaussian_filter

import scenegen
from oracle import geometry, composite, loss, grad, adam, schedule
from oracle.constants import ALPHA_MAX


def test_blur_matches_scipy_gaussian_filter():
    rng = np.random.default_rng(0)
    img = rng.uniform(size=(3, 23, 31))
    got = loss.blur(torch.as_tensor(img)).numpy()
    ref = np.stack([gaussian_filter(img[c], sigma=1.5, truncate=10.0 / 3.0, mode="constant", cval=0.0)
                    for c in range(3)])
    assert np.abs(got - ref).max() < 1e-14


def test_ssim_identity_and_l1_value():
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(3, 20, 17))
    y = rng.uniform(size=(3, 20, 17))
    assert abs(loss.ssim_map(torch.as_tensor(x), torch.as_tensor(x)).mean().item() - 1.0) < 1e-14
    v, g = loss.image_loss_and_grad(x, y, 1.0, 0.0)
    assert abs(v - np.abs(x - y).mean()) < 1e-15
    assert np.abs(g - np.sign(x - y) / x.size).max() < 1e-18


def test_ssim_textbook_and_constant_images():
    """SSIM with the textbook parameters K1 = 0.01, K2 = 0.03, dynamic range L = 1,
    windowed statistics from scipy's Gaussian filter; constant images reduce to
    the luminance term (2ab + C1) / (a^2 + b^2 + C1) away from the border."""
    rng = np.random.default_rng(3)
    x = rng.uniform(size=(3, 25, 22))
    y = np.clip(0.6 * x + 0.3 * rng.uniform(size=x.shape), 0, 1)
    f = lambda im: np.stack([gaussian_filter(im[c], 1.5, truncate=10.0 / 3.0, mode="constant") for c in range(3)])
    c1, c2 = (0.01 * 1.0) ** 2, (0.03 * 1.0) ** 2
    mx, my = f(x), f(y)
    vx, vy, cxy = f(x * x) - mx ** 2, f(y * y) - my ** 2, f(x * y) - mx * my
    ref = ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx ** 2 + my ** 2 + c1) * (vx + vy + c2))
    got = loss.ssim_map(torch.as_tensor(x), torch.as_tensor(y)).numpy()
    assert np.abs(got - ref).max() < 1e-12
    # the loss of one view: w_l1 mean |x - y| + w_dssim (1 - mean SSIM), means over channels and pixels
    val = loss.image_loss(torch.as_tensor(x), torch.as_tensor(y), 0.3, 0.7).item()
    assert val == pytest.approx(0.3 * np.abs(x - y).mean() + 0.7 * (1.0 - ref.mean()), rel=1e-12)
    a, b = 0.2, 0.7
    m = loss.ssim_map(torch.full((1, 20, 20), a, dtype=torch.float64), torch.full((1, 20, 20), b, dtype=torch.float64))
    assert abs(m[0, 10, 10].item() - (2 * a * b + c1) / (a * a + b * b + c1)) < 1e-12


@pytest.mark.parametrize("w_l1,w_dssim", [(0.8, 0.2), (0.0, 1.0)])
def test_loss_gradient_finite_differences(w_l1, w_dssim):
    rng = np.random.default_rng(2)
    x = rng.uniform(size=(3, 14, 12))
    y = rng.uniform(size=(3, 14, 12))
    _, g = loss.image_loss_and_grad(x, y, w_l1, w_dssim)
    h = 1e-6
    for _ in range(40):
        c, j, i = rng.integers(3), rng.integers(14), rng.integers(12)
        if abs(x[c, j, i] - y[c, j, i]) < 10 * h:
            continue
        xp, xm = x.copy(), x.copy()
        xp[c, j, i] += h
        xm[c, j, i] -= h
        fd = (loss.image_loss(torch.as_tensor(xp), torch.as_tensor(y), w_l1, w_dssim).item()
              - loss.image_loss(torch.as_tensor(xm), torch.as_tensor(y), w_l1, w_dssim).item()) / (2 * h)
        assert abs(fd - g[c, j, i]) <= 1e-6 * abs(g).max()


def _structure(params32, n, deg, cams):
    """Discrete structure of a render: visibility, rects, per-pixel lists' ends and
    counts, colour clamps, alpha caps."""
    projs = geometry.project_views(params32, n, deg, cams)
    sig = []
    mins = []
    for p in projs:
        r = composite.render_view(p)
        sig.append((p["visible"].copy(), p["touched"].copy(), r["n_contrib"].copy(), r["last_g"].copy(),
                    (p["rgb_raw"].numpy() < 0).copy()))
        mins.append(min(r["m_cut"].min(), r["m_cap"].min(), r["m_T"].min()))
    return sig, min(mins)


def _same(s1, s2):
    return all(all(np.array_equal(a, b) for a, b in zip(x, y)) for x, y in zip(s1, s2))


def _loss_fd(params32, n, deg, cams, up):
    projs = geometry.project_views(params32, n, deg, cams)
    tot = 0.0
    for p, g in zip(projs, up):
        r = composite.render_view(p, margins=False)
        tot += float((r["color"] * g).sum())
    return tot


@pytest.mark.parametrize("seed,deg,bg", [(41, 3, (0.3, 0.1, 0.6)), (42, 1, (0.0, 0.0, 0.0))])
def test_param_grads_finite_differences(seed, deg, bg):
    """Central differences in FP64 (relative step 1e-6) of L = sum_v <dL/dC_v, C_v>
    agree with the oracle's parameter gradient wherever the discrete structure is
    the same at theta +- h."""
    sc = scenegen.small_scene(seed, 24, deg, [(22, 18), (19, 21)], log_scale_mean=-1.9, bg=bg)
    up = scenegen.upstream_grads(seed + 100, sc.cams, scale=1.0)
    G = grad.param_grads(sc.params, sc.n, deg, sc.cams, up)
    base_sig, _ = _structure(sc.params, sc.n, deg, sc.cams)
    P64 = sc.params[:, :sc.n].astype(np.float64)
    rng = np.random.default_rng(seed)
    checked = 0
    rows = list(range(P64.shape[0]))
    for _ in range(400):
        if checked >= 60:
            break
        r_, g_ = int(rng.choice(rows)), int(rng.integers(sc.n))
        x0 = P64[r_, g_]
        h = 1e-6 * max(1.0, abs(x0))
        vals = []
        ok = True
        for sgn in (+1, -1):
            Q = sc.params.astype(np.float64).copy()
            Q[r_, g_] = x0 + sgn * h
            # the oracle promotes fp32 inputs; feed it FP64 values directly here
            sig, _ = _structure(Q, sc.n, deg, sc.cams)
            if not _same(sig, base_sig):
                ok = False
                break
            vals.append(_loss_fd(Q, sc.n, deg, sc.cams, up))
        if not ok:
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        # truncation error O(h^2) is far below this; the floor is the rounding noise of
        # the two loss evaluations divided by the step
        noise = 64 * np.finfo(np.float64).eps * (abs(vals[0]) + abs(vals[1])) / (2 * h)
        tol = 1e-6 * abs(fd) + noise
        assert abs(fd - G[r_, g_]) <= tol, (r_, g_, fd, G[r_, g_])
        checked += 1
    assert checked >= 40


def test_param_grads_colour_closed_form():
    """For SH degree 0, dL/df_dc = C0 * sum_p dL/dC_p alpha_p T_p (unclamped)."""
    sc = scenegen.small_scene(43, 30, 0, [(20, 16)], log_scale_mean=-1.9)
    up = scenegen.upstream_grads(143, sc.cams, scale=1.0)
    G = grad.param_grads(sc.params, sc.n, 0, sc.cams, up)
    pr = geometry.project_views(sc.params, sc.n, 0, sc.cams)[0]
    # weight alpha*T of Gaussian g at every pixel = colour with unit rgb for g only minus without it
    c0 = 0.5 / math.sqrt(math.pi)
    for g in range(sc.n):
        if not pr["visible"][g] or (pr["rgb_raw"][:, g].numpy() < 0).any():
            continue
        p1 = dict(pr)
        rgb = torch.zeros_like(pr["rgb"])
        rgb[:, g] = 1.0
        p1["rgb"] = rgb
        wgt = composite.render_view(p1, margins=False)["color"][0]
        ref = c0 * (up[0] * wgt[None]).sum(axis=(1, 2))
        assert np.allclose(G[11:14, g], ref, rtol=1e-12, atol=1e-15)


def test_adam_matches_torch_fp64():
    rng = np.random.default_rng(5)
    n_rows, n = 14, 50
    p = rng.normal(size=(n_rows, n))
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    step = np.zeros(n, np.int64)
    lr = [1.6e-4, 5e-3, 1e-3, 2.5e-2, 2.5e-3, 1.25e-4]
    groups = adam.row_groups(n_rows)
    tp = [torch.tensor(p[r], requires_grad=True) for r in range(n_rows)]
    eps = float(np.float32(1e-15))
    opt = torch.optim.Adam([{"params": [tp[r]], "lr": lr[groups[r]]} for r in range(n_rows)],
                           betas=(float(np.float32(0.9)), float(np.float32(0.999))), eps=eps)
    for it in range(5):
        g = rng.normal(size=(n_rows, n))
        p, m, v, step = adam.adam_step(p, g, m, v, step, lr)
        for r in range(n_rows):
            tp[r].grad = torch.tensor(g[r])
        opt.step()
        ref = np.stack([t.detach().numpy() for t in tp])
        assert np.abs(p - ref).max() < 1e-14 * max(1.0, np.abs(ref).max())
    assert (step == 5).all()


def test_adam_view_factor_and_first_step_closed_form():
    n = 6
    p = np.zeros((23, n))
    g = np.ones((23, n))
    vis = np.array([[1, 1, 0, 0, 1, 0], [1, 0, 1, 0, 0, 0], [0, 0, 1, 0, 1, 0]], bool)
    scale = [1.0, 0.5, 0.25]
    lr = [1.0, 2.0, 3.0, 4.0, 5.0, 6.0]
    p1, _, _, _ = adam.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), np.zeros(n, np.int64), lr,
                                 view_scale=scale, visible=vis, group_mask=0b1)
    # first step with a constant gradient: update = lr * 1 / (1 + eps)
    fac = np.array([0.75, 1.0, 0.375, 1.75 / 3, 0.625, 1.75 / 3])
    assert np.allclose(p1[0:3], -fac[None, :], rtol=1e-12)
    assert np.allclose(p1[3:6], -2.0, rtol=1e-12) and np.allclose(p1[14], -6.0, rtol=1e-12)


def test_adam_group_rates_follow_the_parameter_layout():
    # Every row's first step with a constant gradient moves it by its group's rate
    # (update = lr / (1 + eps)); the groups follow the parameter layout: mean rows
    # 0-2, log-scale 3-5, quaternion 6-9, opacity 10, SH coefficient 0 (the DC
    # term, three channels) 11-13, the other SH coefficients after them.
    lr = [1.0, 2.0, 3.0, 4.0, 5.0, 6.0]
    for deg in range(4):
        rows = 11 + 3 * (deg + 1) ** 2
        want = np.empty(rows)
        want[0:3], want[3:6], want[6:10], want[10] = lr[0], lr[1], lr[2], lr[3]
        for k in range((deg + 1) ** 2):
            want[11 + 3 * k: 14 + 3 * k] = lr[4] if k == 0 else lr[5]
        n = 3
        p1, _, _, _ = adam.adam_step(np.zeros((rows, n)), np.ones((rows, n)), np.zeros((rows, n)),
                                     np.zeros((rows, n)), np.zeros(n, np.int64), lr)
        assert np.allclose(-p1, want[:, None], rtol=1e-12), deg


def test_schedule_eq6_to_eq8():
    e0, ef, ta = 1.6e-4, 1.6e-6, 200
    assert schedule.lr_current(0, e0, ef, ta) == pytest.approx(e0, rel=1e-15)
    assert schedule.lr_current(ta, e0, ef, ta) == pytest.approx(ef, rel=1e-15)
    assert schedule.lr_current(10 * ta, e0, ef, ta) == pytest.approx(ef, rel=1e-15)
    mid = schedule.lr_current(ta / 2, e0, ef, ta)
    assert mid == pytest.approx(math.sqrt(e0 * ef), rel=1e-14)      # geometric interpolation
    M = np.array([[0, 0.5, 0], [0.5, 0, 0.2], [0, 0.2, 0]])
    lrs = [1.0, 2.0, 4.0]
    assert schedule.lr_neighbourhood(1, lrs, M) == pytest.approx((2.0 + 0.5 * 1.0 + 0.2 * 4.0) / 3)
    assert schedule.lr_neighbourhood(0, lrs, M) == pytest.approx((1.0 + 0.5 * 2.0) / 2)


def test_schedule_eq3_to_eq5():
    # chain 3 - 2 - 1 - 0 (new = 3) plus 4 attached to both 2 and 1
    M = np.zeros((5, 5))
    for i, j, wgt in [(3, 2, 0.8), (2, 1, 0.5), (1, 0, 0.6), (4, 2, 0.4), (4, 1, 0.3)]:
        M[i, j] = M[j, i] = wgt
    w = schedule.hierarchical_weights(M, 3)
    assert w[3] == 1.0 and w[2] == pytest.approx(0.8)
    assert w[1] == pytest.approx(0.8 * 0.5) and w[4] == pytest.approx(0.8 * 0.4)
    assert w[0] == pytest.approx((0.4 * 0.6 + 0.32 * 0.0) / 2)
    b = schedule.local_budget(w, 3, 200)
    assert sum(b.values()) == 100 and set(b) == {3, 2, 1} or set(b) == {3, 2, 4}
    raw = {i: 1 - math.exp(-w[i]) for i in b}
    for i in b:
        assert abs(b[i] - raw[i] / (2 * sum(raw.values())) * 200) < 1.0


def test_schedule_iteration_plan():
    """Plan pins: local counts are Eq. 5's shares, the semi-global half is spread
    evenly (counts differ by <= 1) over the non-key images, draws without
    replacement when they outnumber the iterations, and hand-worked small case."""
    M = np.array([[0, .5, 0, 0], [.5, 0, .2, 0], [0, .2, 0, 0], [0, 0, 0, 0]], float)
    w = schedule.hierarchical_weights(M, 0)
    # shares of Eq. 5 at T_I = 10 over the top 2 (images 0, 1): 3.08 -> 3, 1.92 -> 2
    assert schedule.iteration_plan(w, 4, 2, 10, [.3, .1, .2, .05]) == [0, 1, 0, 1, 0, 3, 2, 3, 2, 3]
    rng = np.random.default_rng(7)
    n = 60
    A = (rng.random((n, n)) < 0.08) * rng.random((n, n))
    A = np.maximum(A, A.T)
    np.fill_diagonal(A, 0)
    w = schedule.hierarchical_weights(A, 5)
    u = rng.random(n)
    plan = schedule.iteration_plan(w, n, 10, 200, u)
    assert len(plan) == 200
    share = schedule.local_budget(w, 10, 200)
    local = plan[:100]
    assert {i: local.count(i) for i in share} == share
    semi = plan[100:]
    others = [i for i in range(n) if i not in share]
    cnt = np.array([semi.count(i) for i in others])
    assert cnt.sum() == 100 and cnt.max() - cnt.min() <= 1 and not set(semi) & set(share)
    # more remaining images than iterations: no repeats
    plan = schedule.iteration_plan(w, n, 10, 20, u)
    assert len(set(plan[10:])) == 10
    # a lone image takes every iteration
    assert schedule.iteration_plan({0: 1.0}, 1, 10, 7, [0.5]) == [0] * 7



def test_load_balance_loss_eq9():
    """Eq. 9 pins: population std (numpy), two-valued closed form, zero for a
    constant map with zero gradient, and central differences of the gradient."""
    rng = np.random.default_rng(3)
    G = rng.random((7, 9)) * 3.0
    val, g = loss.load_balance_loss_and_grad(G)
    assert val == pytest.approx(float(np.std(G)), rel=1e-14)
    half = np.zeros((4, 6))
    half[:, :3] = 1.0
    v2, g2 = loss.load_balance_loss_and_grad(half)
    assert v2 == pytest.approx(0.5, rel=1e-15)
    assert np.allclose(g2, (half - 0.5) / (half.size * 0.5), rtol=1e-14)
    v0, g0 = loss.load_balance_loss_and_grad(np.full((3, 3), 2.5))
    assert v0 == 0.0 and not g0.any()
    h = 1e-6
    for (j, i) in [(0, 0), (3, 4), (6, 8)]:
        Gp, Gm = G.copy(), G.copy()
        Gp[j, i] += h
        Gm[j, i] -= h
        fd = (np.std(Gp) - np.std(Gm)) / (2 * h)
        assert abs(fd - g[j, i]) <= 1e-8


def test_param_grads_with_load_term_finite_differences():
    """The gradient of L = <dL/dC, C> + <dL/dA, alpha_sum> (load-balancing upstream
    on the soft count) agrees with central differences of the oracle forward."""
    sc = scenegen.small_scene(47, 24, 1, [(22, 18)], log_scale_mean=-1.9)
    up = scenegen.upstream_grads(147, sc.cams, scale=1.0)
    rng = np.random.default_rng(47)
    upA = [rng.normal(0, 1, size=(c["height"], c["width"])) for c in sc.cams]
    G = grad.param_grads(sc.params, sc.n, 1, sc.cams, up, dL_dalpha_sum=upA)
    G0 = grad.param_grads(sc.params, sc.n, 1, sc.cams, up)
    assert np.abs(G - G0).max() > 1e-3 * np.abs(G0).max()      # the load term moves the gradient

    def obj(Q):
        tot = 0.0
        for c, g, gA in zip(sc.cams, up, upA):
            p = geometry.project_view(torch.as_tensor(Q), c, 1)
            r = composite.render_view(p, margins=False)
            tot += float((r["color"] * g).sum()) + float((r["alpha_sum"] * gA).sum())
        return tot

    base_sig, _ = _structure(sc.params, sc.n, 1, sc.cams)
    checked = 0
    for _ in range(300):
        if checked >= 30:
            break
        r_, g_ = int(rng.integers(sc.params.shape[0])), int(rng.integers(sc.n))
        x0 = float(sc.params[r_, g_])
        h = 1e-6 * max(1.0, abs(x0))
        vals = []
        for sgn in (+1, -1):
            Q = sc.params.astype(np.float64).copy()
            Q[r_, g_] = x0 + sgn * h
            sig, _ = _structure(Q, sc.n, 1, sc.cams)
            if not _same(sig, base_sig):
                vals = None
                break
            vals.append(obj(Q[:, :sc.n]))
        if vals is None:
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        noise = 64 * np.finfo(np.float64).eps * (abs(vals[0]) + abs(vals[1])) / (2 * h)
        assert abs(fd - G[r_, g_]) <= 1e-6 * abs(fd) + noise, (r_, g_, fd, G[r_, g_])
        checked += 1
    assert checked >= 20
