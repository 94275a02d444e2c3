"""Differentiation at scale (3M Gaussians, SH degree 3, one 1920x1080 view): the
autograd backward of the whole field against the FP64 oracle gradient of a ~2k
Gaussian crop, against central finite differences of the oracle forward on 64
parameters, and the context memory of stored vs recomputed forward state."""
import numpy as np
import pytest
import torch

import scenegen
import oracle
from oracle import composite
from oracle.geometry import params_f64, project_view
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

# a 16x16 window: at this density the Gaussians whose rects meet it number ~2k
X0, Y0, S = 400, 300, 16


@pytest.fixture(scope="module")
def c4():
    sc = scenegen.config4()
    cam = sc.cams[0]
    P64 = params_f64(sc.params, sc.n)
    with torch.no_grad():
        p = project_view(P64, cam, sc.sh_degree)
    hit = (p["touched"] > 0) & (p["i0"] <= X0 + S - 1) & (p["i1"] >= X0) & (p["j0"] <= Y0 + S - 1) & (p["j1"] >= Y0)
    crop = np.nonzero(hit)[0]
    del P64, p
    Pc = np.ascontiguousarray(sc.params[:, crop])
    pc = project_view(params_f64(Pc, len(crop)), cam, sc.sh_degree)
    yy, xx = np.mgrid[Y0:Y0 + S, X0:X0 + S]
    r = composite.composite_pixels(pc, xx.ravel(), yy.ravel(), margins=True)
    amb = gu.ambiguous(r)
    rng = np.random.default_rng(44)
    w = np.zeros((3, cam["height"], cam["width"]), np.float32)
    w[:, Y0:Y0 + S, X0:X0 + S] = rng.normal(0, 1, size=(3, S, S))
    w[:, yy.ravel()[amb], xx.ravel()[amb]] = 0.0
    return dict(sc=sc, cam=cam, crop=crop, Pc=Pc, w=w, n_amb=int(amb.sum()), r=r)


def _gpu_grad(sc, cam, w, mode="store"):
    from paper_2503_13086_amd.autograd import rasterize
    P = torch.as_tensor(sc.params).cuda().requires_grad_(True)
    img = rasterize(P, sc.n, sc.sh_degree, [cam], mode=mode)
    (img * torch.as_tensor(w).reshape(-1).cuda()).sum().backward()
    g = P.grad.cpu().numpy()
    del P, img
    return g


def test_c4_crop_gradient_matches_oracle(c4):
    sc, cam, crop, w = c4["sc"], c4["cam"], c4["crop"], c4["w"]
    assert 1000 <= len(crop) <= 4000 and c4["n_amb"] <= S * S // 50
    g = _gpu_grad(sc, cam, w)
    outside = np.ones(sc.n, bool)
    outside[crop] = False
    assert not g[:, outside].any()                    # only the crop can reach the window
    ref = oracle.param_grads(c4["Pc"], len(crop), sc.sh_degree, [cam], [w])
    errs = gu.grad_errors(g[:, crop], ref, np.ones(len(crop), bool), gu.param_groups(sc.sh_degree))
    for name, (rel, elem) in errs.items():
        assert rel <= 1e-3 and elem <= 1.0, (name, rel, elem)


def test_c4_finite_differences(c4):
    """h = 1e-4 central differences of the FP64 oracle forward on the crop (window
    pixels only, where the blend structure is unchanged by the step) against the
    GPU gradient of the full field."""
    sc, cam, crop, w, Pc = c4["sc"], c4["cam"], c4["crop"], c4["w"], c4["Pc"]
    g = _gpu_grad(sc, cam, w)[:, crop]
    yy, xx = np.mgrid[Y0:Y0 + S, X0:X0 + S]
    px, py = xx.ravel(), yy.ravel()
    wv = w[:, py, px].astype(np.float64)
    base = Pc.astype(np.float64)
    r0 = c4["r"]
    rng = np.random.default_rng(5)
    cand = np.nonzero(np.abs(g).max(axis=0) > 0)[0]
    checked = 0
    for _ in range(600):
        if checked >= 64:
            break
        col = int(rng.choice(cand))
        row = int(rng.integers(base.shape[0]))
        h = 1e-4 * max(1.0, abs(base[row, col]))
        vals = []
        for sgn in (1, -1):
            Q = base.copy()
            Q[row, col] += sgn * h
            with torch.no_grad():
                pr = project_view(torch.as_tensor(Q), cam, sc.sh_degree)
            rr = composite.composite_pixels(pr, px, py, margins=False)
            if not (np.array_equal(rr["n_contrib"], r0["n_contrib"]) and np.array_equal(rr["last_g"], r0["last_g"])):
                vals = None
                break
            vals.append(float((rr["color"] * wv).sum()))
        if vals is None:
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[row, col]) <= 2e-3 * abs(fd) + 1e-3 * np.abs(g[row]).max() + 1e-6, (row, col, fd,
                                                                                              g[row, col])
        checked += 1
    assert checked >= 48


def test_c4_store_vs_recompute_memory(c4):
    """Two forwards awaiting their backward: stored state keeps one context per
    forward, recomputation keeps one shared context; the gradients agree."""
    from paper_2503_13086_amd.autograd import rasterize, context_bytes
    sc, cam = c4["sc"], c4["cam"]
    rng = np.random.default_rng(8)
    cams = [cam, dict(cam, t=np.asarray(cam["t"], np.float32) + np.float32([0.3, 0.0, 0.0]))]
    ws = [torch.as_tensor(rng.normal(0, 1e-3, size=3 * cam["width"] * cam["height"]).astype(np.float32)).cuda()
          for _ in cams]
    res = {}
    for mode in ("store", "recompute"):
        base = context_bytes()
        P = torch.as_tensor(sc.params).cuda().requires_grad_(True)
        imgs = [rasterize(P, sc.n, sc.sh_degree, [c], mode=mode) for c in cams]
        held = context_bytes() - base
        sum((im * wv).sum() for im, wv in zip(imgs, ws)).backward()
        res[mode] = (held, P.grad.cpu().numpy())
        del P, imgs
    print(f"context bytes with two pending forwards: store {res['store'][0] / 2**20:.1f} MiB, "
          f"recompute {res['recompute'][0] / 2**20:.1f} MiB")
    assert res["recompute"][0] < 0.6 * res["store"][0]
    g1, g2 = res["store"][1], res["recompute"][1]
    assert np.abs(g1 - g2).max() <= 1e-5 * np.abs(g1).max()
