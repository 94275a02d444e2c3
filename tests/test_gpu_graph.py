"""A whole training step (gs_preprocess, gs_bin_sort without waiting, gs_render_fwd,
gs_loss, gs_render_bwd_adam) captured into a HIP graph and replayed: every replay,
with eager work between replays, matches an eager step from the same state (image
and loss bit for bit, gradient within the parity bar, and its parameters, moments
and step counters those of the oracle's Adam step applied to the gradient the
replay wrote).  Calls that would allocate or wait during capture are refused."""
import numpy as np
import pytest
import torch

import scenegen
import oracle
import paper_2503_13086_amd as gs
from paper_2503_13086_amd.pipeline import Rasterizer, params_to_device, DEFAULT_LR
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _state(P):
    return dict(P=P.clone(), m=torch.zeros_like(P), v=torch.zeros_like(P),
                step=torch.zeros(P.shape[1], dtype=torch.int32, device=P.device))


def _step(rz, st, sc, target, color, dl, loss, G):
    rz.preprocess(st["P"], sc.n, sc.sh_degree, sc.cams)
    rz.bin_sort(count=False)
    rz.render_fwd(color)
    rz.loss(color, target, sc.w_l1, sc.w_dssim, loss, dl)
    rz.render_bwd_adam(dl, st["m"], st["v"], st["step"], DEFAULT_LR, [1.0, 0.5], group_mask=1, grad=G)


def test_captured_step_replays_like_eager_steps():
    sc = scenegen.small_scene(301, 2000, 1, [(96, 64), (80, 72)], log_scale_mean=-2.6, w_l1=0.8, w_dssim=0.2)
    P0 = params_to_device(sc.params)
    rz_e, rz_g = Rasterizer(0), Rasterizer(0)
    try:
        bufs = {}
        for name, rz in (("e", rz_e), ("g", rz_g)):
            rz.set_views(sc.cams)
            bufs[name] = dict(st=_state(P0), color=rz.new_image(), dl=rz.new_image(),
                              loss=torch.zeros(2, dtype=torch.float64, device=P0.device), G=torch.zeros_like(P0),
                              target=rz.pack_images(sc.targets))
        for name, rz in (("e", rz_e), ("g", rz_g)):   # uncaptured steps size every buffer
            b = bufs[name]
            rz.preprocess(b["st"]["P"], sc.n, sc.sh_degree, sc.cams)
            rz.bin_sort(count=True)
            for _ in range(2):
                _step(rz, b["st"], sc, b["target"], b["color"], b["dl"], b["loss"], b["G"])
        torch.cuda.synchronize()
        be, bg = bufs["e"], bufs["g"]
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            _step(rz_g, bg["st"], sc, bg["target"], bg["color"], bg["dl"], bg["loss"], bg["G"])
        torch.cuda.synchronize()
        for it in range(3):
            # the replay and the eager step start from the same state
            for k in ("P", "m", "v", "step"):
                bg["st"][k].copy_(be["st"][k])
            pre = {k: t.cpu().numpy().copy() for k, t in be["st"].items()}
            graph.replay()
            _step(rz_e, be["st"], sc, be["target"], be["color"], be["dl"], be["loss"], be["G"])
            torch.cuda.synchronize()
            print(f"[graph] replay {it}: loss {bg['loss'].cpu().numpy()}", flush=True)
            assert torch.equal(bg["color"], be["color"]), it
            assert torch.equal(bg["loss"], be["loss"]), it
            Gg, Ge = bg["G"][:, :sc.n].cpu().numpy(), be["G"][:, :sc.n].cpu().numpy()
            errs = gu.grad_errors(Gg, Ge, np.ones(sc.n, bool), gu.param_groups(sc.sh_degree))
            for grp, (rel, elem) in errs.items():
                assert rel <= 1e-5 and elem <= 1.0, (it, grp, rel, elem)
            vis = (rz_g.buffer(gs.GS_BUF_TOUCHED).view(2, sc.n) > 0).cpu().numpy()
            p1, m1, v1, s1 = oracle.adam_step(pre["P"], Gg, pre["m"], pre["v"], pre["step"].view(np.uint32),
                                              DEFAULT_LR, view_scale=[1.0, 0.5], visible=vis, group_mask=1)
            out = {k: t.cpu().numpy() for k, t in bg["st"].items()}
            assert np.array_equal(out["step"].astype(np.int64), s1)
            assert np.abs(out["m"] - m1).max() <= 1e-6 * np.abs(m1).max()
            assert np.abs(out["v"] - v1).max() <= 1e-6 * np.abs(v1).max()
            dp_ref, dp = p1 - pre["P"], out["P"].astype(np.float64) - pre["P"]
            assert np.all(np.abs(dp - dp_ref) <= 1e-4 * np.abs(dp_ref) + 2 * np.spacing(np.abs(pre["P"]))), it
        rz_g.sync_status()
        # under capture, a call that would wait for K is refused (and the capture discarded)
        with pytest.raises(Exception):
            g2 = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g2):
                rz_g.preprocess(bg["st"]["P"], sc.n, sc.sh_degree, sc.cams)
                rz_g.bin_sort(count=True)
        torch.cuda.synchronize()
    finally:
        rz_e.close()
        rz_g.close()
