"""The ordered backward (gs_set_backward_order(GS_BWD_ORDERED)), through the C ABI:
every Gaussian's per-tile partial sums added in tile order instead of by
floating-point atomics.  Its 2D and parameter gradients, and the parameters and
moments of a fused backward + Adam step, are the same bits on every run; they
differ from the atomic order's by rounding only; and they meet the same bar
against the FP64 oracle (Sec. IV-E splat-level accumulation; Sec. IV-D Adam)."""
import numpy as np
import pytest
import torch

import scenegen
import oracle
from oracle import composite
import paper_2503_13086_amd as gs
from paper_2503_13086_amd.pipeline import Rasterizer, params_to_device
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _scene():
    # splats of tens of pixels over two views of uneven size: most Gaussians add
    # partials from several tiles, so the atomic order varies between runs
    return scenegen.small_scene(301, 2500, 2, [(160, 120), (112, 96)], log_scale_mean=-2.2, w_l1=0.8, w_dssim=0.2)


_cache = {}


def _upstream(sc):
    if "up" not in _cache:
        projs = oracle.project_views(sc.params, sc.n, sc.sh_degree, sc.cams)
        renders = [composite.render_view(p) for p in projs]
        up = gu.masked_upstream(scenegen.upstream_grads(11, sc.cams, scale=1e-2), [gu.ambiguous(r) for r in renders])
        _cache["up"] = (up, projs)
    return _cache["up"]


@pytest.mark.parametrize("tile", [16, 8, 32])
def test_ordered_backward_is_the_same_bits_every_run(tile):
    sc = _scene()
    up, _ = _upstream(sc)
    runs = [gu.run_gpu(sc, upstream=up, tile=tile, bwd="ordered") for _ in range(3)]
    tiles_per_gaussian = np.count_nonzero(runs[0]["grad2d"].reshape(-1, 9).any(1))
    print(f"[ordered] tile {tile}: {tiles_per_gaussian} (view, Gaussian) entries with a gradient", flush=True)
    for r in runs[1:]:
        assert np.array_equal(r["grad2d"].view(np.uint32), runs[0]["grad2d"].view(np.uint32))
        assert np.array_equal(r["grad"].view(np.uint32), runs[0]["grad"].view(np.uint32))


def test_ordered_backward_matches_atomic_to_rounding():
    sc = _scene()
    up, _ = _upstream(sc)
    ga = gu.run_gpu(sc, upstream=up, bwd="atomic")
    go = gu.run_gpu(sc, upstream=up, bwd="ordered")
    ga2 = gu.run_gpu(sc, upstream=up, bwd="atomic")
    print(f"[ordered] two atomic runs differ in {int((ga['grad2d'] != ga2['grad2d']).sum())} of "
          f"{ga['grad2d'].size} 2D gradient values", flush=True)
    a2, o2 = ga["grad2d"].reshape(-1, 9), go["grad2d"].reshape(-1, 9)
    scale = np.abs(a2).max(0) + 1e-30
    assert (np.abs(a2 - o2) / scale).max() <= 1e-5
    for grp, rows in gu.param_groups(sc.sh_degree).items():
        a, o = ga["grad"][rows], go["grad"][rows]
        assert np.linalg.norm(a - o) <= 1e-5 * (np.linalg.norm(a) + 1e-30), grp


def test_ordered_backward_against_the_oracle():
    sc = _scene()
    up, _ = _upstream(sc)
    g = gu.run_gpu(sc, upstream=up, bwd="ordered")
    ref = oracle.param_grads(sc.params, sc.n, sc.sh_degree, sc.cams, up)
    errs = gu.grad_errors(g["grad"], ref, np.ones(sc.n, bool), gu.param_groups(sc.sh_degree))
    for grp, (rel, elem) in errs.items():
        assert rel <= 1e-3 and elem <= 1.0, (grp, rel, elem)


def test_ordered_fused_adam_is_the_same_bits_every_run():
    """Five training steps of forward, loss and fused backward + Adam from the same
    state: parameters, moments and step counts agree bit for bit between runs."""
    sc = _scene()
    start = params_to_device(sc.params).cpu().numpy().copy()
    outs = []
    for _ in range(2):
        rz = Rasterizer(0)
        try:
            gs.gs_set_backward_order(rz.ctx, gs.GS_BWD_ORDERED)
            P = params_to_device(sc.params)
            m, v = torch.zeros_like(P), torch.zeros_like(P)
            step = torch.zeros(sc.n, dtype=torch.int32, device=P.device)
            rz.set_views(sc.cams)
            tgt = rz.pack_images(sc.targets)
            for _ in range(5):
                rz.preprocess(P, sc.n, sc.sh_degree)
                rz.bin_sort()
                color = rz.render_fwd()
                _, dl = rz.loss(color, tgt, sc.w_l1, sc.w_dssim)
                rz.render_bwd_adam(dl, m, v, step, view_lr_scale=[1.0, 0.5])
            rz.sync_status()
            torch.cuda.synchronize()
            outs.append([x.cpu().numpy().copy() for x in (P, m, v, step)])
        finally:
            rz.close()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert not np.array_equal(outs[0][0], start) and int(outs[0][3].max()) == 5


def test_ordered_backward_with_the_load_balancing_term():
    """The Eq. 9 gradient (added to every blended alpha's derivative) goes through
    the ordered backward as through the atomic one: the two agree to rounding and
    the ordered one is the same bits on a second run."""
    sc = _scene()
    outs = {}
    for mode, runs in ((gs.GS_BWD_ATOMIC, 1), (gs.GS_BWD_ORDERED, 2)):
        for r in range(runs):
            rz = Rasterizer(0)
            try:
                gs.gs_set_backward_order(rz.ctx, mode)
                P = params_to_device(sc.params)
                rz.preprocess(P, sc.n, sc.sh_degree, sc.cams)
                rz.bin_sort()
                color = rz.render_fwd()
                _, dl = rz.loss(color, rz.pack_images(sc.targets), 0.47, 0.12)
                rz.load_balance(0.41)
                grad = rz.render_bwd(dl)
                torch.cuda.synchronize()
                outs[(mode, r)] = grad[:, : sc.n].cpu().numpy().copy()
            finally:
                rz.close()
    a, o1, o2 = outs[(gs.GS_BWD_ATOMIC, 0)], outs[(gs.GS_BWD_ORDERED, 0)], outs[(gs.GS_BWD_ORDERED, 1)]
    assert np.array_equal(o1.view(np.uint32), o2.view(np.uint32))
    for grp, rows in gu.param_groups(sc.sh_degree).items():
        assert np.linalg.norm(a[rows] - o1[rows]) <= 1e-5 * (np.linalg.norm(a[rows]) + 1e-30), grp
    assert np.abs(a).max() > 0


def test_unknown_backward_order_is_refused():
    rz = Rasterizer(0)
    try:
        with pytest.raises(gs.GsError) as ei:
            gs.gs_set_backward_order(rz.ctx, 7)
        assert ei.value.status == gs.GS_ERR_INVALID
    finally:
        rz.close()
