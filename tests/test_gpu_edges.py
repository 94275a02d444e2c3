"""Edge and degenerate cases of the HIP path (through the C ABI) against the oracle,
and the argument checks of every entry point."""
import numpy as np
import pytest
import torch

import scenegen
import oracle
from oracle import composite
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _one_gaussian(z=3.0, ls=-2.0, rho=2.0, size=(1, 1), bg=(0.25, 0.5, 0.75)):
    P = np.zeros((14, 1), np.float32)
    P[2, 0] = z
    P[3:6, 0] = ls
    P[6, 0] = 1.0
    P[10, 0] = rho
    P[11:14, 0] = [1.0, -0.5, 0.3]
    W, H = size
    cam = scenegen.camera(np.eye(3), np.zeros(3), 50.0, 50.0, W / 2, H / 2, W, H, bg)
    return scenegen.Scene(P, 1, 0, [cam], [np.zeros((3, H, W), np.float32)])


@pytest.mark.parametrize("size", [(1, 1), (17, 1), (1, 33), (16, 16), (31, 17)])
def test_single_gaussian_tiny_images(size):
    sc = _one_gaussian(size=size)
    p = oracle.project_views(sc.params, 1, 0, sc.cams)
    g = gu.run_gpu(sc, upstream=[np.ones((3, size[1], size[0]), np.float32)])
    r = composite.render_view(p[0])
    assert np.abs(g["color"][0] - r["color"]).max() <= 1e-5
    ref = oracle.param_grads(sc.params, 1, 0, sc.cams, [np.ones((3, size[1], size[0]))])
    assert np.abs(g["grad"] - ref).max() <= 1e-4 * max(1e-6, np.abs(ref).max())


def test_nothing_visible():
    """Every Gaussian behind the camera: no pairs, image = background, zero grads."""
    sc = scenegen.small_scene(3, 200, 1, [(40, 30), (20, 20)], bg=(0.3, 0.6, 0.9))
    sc.params[2, :] = -50.0       # far behind both cameras (cameras sit at z ~ -3 looking at +z)
    sc.params[0:2, :] = 0.0
    g = gu.run_gpu(sc, upstream=scenegen.upstream_grads(1, sc.cams))
    assert g["K"] == 0
    for v, c in enumerate(sc.cams):
        assert np.allclose(g["color"][v], np.asarray(c["bg"], np.float32)[:, None, None])
    assert (g["T_final"] == 1.0).all() and (g["n_contrib"] == 0).all()
    assert (g["grad"] == 0).all()


def test_near_plane_and_offscreen():
    """Gaussians straddling the near plane and far off-screen are culled exactly as
    the oracle culls them; large ones overlapping the border are kept."""
    rng = np.random.default_rng(4)
    n = 600
    P = scenegen.make_field(rng, n, 0, center=(0, 0, 0.5), half_extent=2.0, log_scale_mean=-1.5)
    P[2, :200] = rng.uniform(0.15, 0.25, 200)          # around the near plane (0.2)
    cam = scenegen.camera(np.eye(3), np.zeros(3), 60.0, 60.0, 32.0, 24.0, 64, 48)
    sc = scenegen.Scene(P, n, 0, [cam], [np.zeros((3, 48, 64), np.float32)])
    projs = oracle.project_views(P, n, 0, [cam])
    g = gu.run_gpu(sc)
    assert np.array_equal(g["touched"][0], projs[0]["touched"])
    b = oracle.bin_pairs(projs, [cam], 16)
    keys, values, _ = gu.valid_pairs(g)
    assert np.array_equal(keys, b["keys"]) and np.array_equal(values, b["values"])
    r = composite.render_view(projs[0])
    ok = ~gu.ambiguous(r)
    assert np.abs(g["color"][0] - r["color"]).max(axis=0)[ok].max() <= 1e-4


def test_stride_larger_than_n_and_accumulate():
    """Columns beyond n are never read or written; accumulate adds to grad."""
    from paper_2503_13086_amd.pipeline import Rasterizer
    sc = scenegen.small_scene(8, 300, 2, [(48, 40)])
    stride = 512
    P = np.full((sc.params.shape[0], stride), np.nan, np.float32)
    P[:, :sc.n] = sc.params[:, :sc.n]
    up = scenegen.upstream_grads(2, sc.cams)
    rz = Rasterizer(0)
    try:
        tP = torch.as_tensor(P).cuda()
        rz.preprocess(tP, sc.n, 2, sc.cams)
        rz.bin_sort()
        rz.render_fwd()
        grad = torch.full_like(tP, 7.0)
        rz.render_bwd(rz.pack_images(up), grad, accumulate=True)
        g = grad.cpu().numpy()
    finally:
        rz.close()
    assert (g[:, sc.n:] == 7.0).all()
    ref = oracle.param_grads(sc.params, sc.n, 2, sc.cams, up)
    assert np.abs((g[:, :sc.n] - 7.0) - ref).max() <= 1e-3 * np.abs(ref).max() + 1e-6


def test_batched_equals_plain_loop():
    """Rendering three views in one batch equals three single-view calls (images
    bit for bit, gradients summed over views within fp32 atomics)."""
    from paper_2503_13086_amd.pipeline import Rasterizer, params_to_device
    sc = scenegen.small_scene(12, 1500, 3, [(70, 50), (33, 64), (90, 20)], log_scale_mean=-2.6)
    up = scenegen.upstream_grads(5, sc.cams, 1e-2)
    rz = Rasterizer(0)
    try:
        P = params_to_device(sc.params)
        rz.preprocess(P, sc.n, 3, sc.cams)
        rz.bin_sort()
        col = rz.render_fwd()
        imgs = [x.clone() for x in rz.image_views(col)]
        gb = rz.render_bwd(rz.pack_images(up))
        gl = torch.zeros_like(P)
        singles = []
        for v, c in enumerate(sc.cams):
            rz.preprocess(P, sc.n, 3, [c])
            rz.bin_sort()
            singles.append(rz.render_fwd().view(3, c["height"], c["width"]).clone())
            rz.render_bwd(rz.pack_images([up[v]]), gl, accumulate=True)
        for a, b in zip(imgs, singles):
            assert torch.equal(a, b)
        gb, gl = gb.cpu().numpy(), gl.cpu().numpy()
    finally:
        rz.close()
    assert np.abs(gb - gl).max() <= 1e-5 * np.abs(gb).max()


def test_argument_checks():
    import paper_2503_13086_amd as gs
    from paper_2503_13086_amd.pipeline import Rasterizer
    sc = scenegen.small_scene(1, 10, 0, [(16, 16)])
    rz = Rasterizer(0)
    try:
        P = torch.as_tensor(sc.params).cuda()
        rz.set_views(sc.cams)
        with pytest.raises(gs.GsError) as e:
            gs.gs_bin_sort(rz.ctx)
        assert e.value.status == gs.GS_ERR_STATE
        with pytest.raises(gs.GsError) as e:
            gs.gs_preprocess(rz.ctx, P, 10, 5, 0, sc.cams)            # stride < n
        assert e.value.status == gs.GS_ERR_INVALID
        with pytest.raises(gs.GsError) as e:
            gs.gs_preprocess(rz.ctx, P, 10, 10, 4, sc.cams)           # SH degree 4
        assert e.value.status == gs.GS_ERR_INVALID
        with pytest.raises(gs.GsError) as e:
            gs.gs_preprocess(rz.ctx, P, 10, 10, 0, sc.cams, tile=12)
        assert e.value.status == gs.GS_ERR_UNSUPPORTED
        bad = dict(sc.cams[0])
        bad["fx"] = 0.0
        with pytest.raises(gs.GsError) as e:
            gs.gs_preprocess(rz.ctx, P, 10, 10, 0, [bad])
        assert e.value.status == gs.GS_ERR_INVALID
        with pytest.raises(gs.GsError) as e:
            gs.gs_preprocess(rz.ctx, P, 10, 10, 0, sc.cams * 65)      # too many views
        assert e.value.status == gs.GS_ERR_INVALID
        with pytest.raises(gs.GsError) as e:
            gs.gs_preprocess(rz.ctx, P.data_ptr() + 2, 10, 10, 0, sc.cams)   # misaligned
        assert e.value.status == gs.GS_ERR_INVALID
        gs.gs_preprocess(rz.ctx, P, 10, 10, 0, sc.cams)
        with pytest.raises(gs.GsError) as e:
            gs.gs_render_fwd(rz.ctx, rz.new_image())                   # before bin_sort
        assert e.value.status == gs.GS_ERR_STATE
        with pytest.raises(gs.GsError) as e:
            gs.gs_adam_step(rz.ctx, P, P, P, P, torch.zeros(10, dtype=torch.int32).cuda(), 10, 10, 0,
                            [1e-3] * 6, [1.0, 1.0], beta1=0.9)             # 2 view scales, 1 view
        assert e.value.status == gs.GS_ERR_STATE
        assert "n_views" in gs.gs_last_error(rz.ctx)
        S = torch.zeros(10, dtype=torch.int32).cuda()
        img = rz.new_image(0.0)
        with pytest.raises(gs.GsError) as e:
            gs.gs_render_bwd_adam(rz.ctx, P, img, None, P, P, S, [1e-3] * 6)   # before render_fwd
        assert e.value.status == gs.GS_ERR_STATE
        rz.preprocess(P, 10, 0)
        rz.bin_sort()
        rz.render_fwd()
        with pytest.raises(gs.GsError) as e:
            gs.gs_render_bwd_adam(rz.ctx, P, img, None, None, P, S, [1e-3] * 6)   # m missing
        assert e.value.status == gs.GS_ERR_INVALID
        with pytest.raises(gs.GsError) as e:
            gs.gs_render_bwd_adam(rz.ctx, P, img, P.data_ptr() + 2, P, P, S, [1e-3] * 6)   # misaligned grad
        assert e.value.status == gs.GS_ERR_INVALID
        with pytest.raises(gs.GsError) as e:
            gs.gs_render_bwd_adam(rz.ctx, P, img, None, P, P, S, [1e-3] * 6, beta1=1.0)
        assert e.value.status == gs.GS_ERR_INVALID
        with pytest.raises(gs.GsError) as e:
            gs.gs_render_bwd_adam(rz.ctx, P, img, None, P, P, S, [1e-3] * 6, [1.0, 1.0])   # 2 scales, 1 view
        assert e.value.status == gs.GS_ERR_STATE
    finally:
        rz.close()


def test_bin_sort_counts_past_255():
    """Gaussians spanning hundreds of tiles: per-entry pair counts above 255 (the
    depth sort's values carry counts only up to 255; larger ones are read back from
    the per-entry array), and emission waves (64 depth-ordered entries) holding more
    entries of over 64 candidate tiles than emission keeps in LDS (8; the rest re-derive
    their test geometry from the record).  Keys, values and ranges bit-exact against
    the oracle."""
    sc = scenegen.small_scene(21, 120, 0, [(1024, 768)], log_scale_mean=-1.2)
    projs = oracle.project_views(sc.params, sc.n, 0, sc.cams)
    b = oracle.bin_pairs(projs, sc.cams, 16, cull="ellipse")
    per_g = np.bincount(b["values"].astype(np.int64), minlength=sc.n)
    assert per_g.max() > 255 and (per_g > 0).sum() >= 50
    p0 = projs[0]
    vis = np.nonzero(p0["visible"])[0]
    order = vis[np.lexsort((vis, p0["depth_bits"][vis]))]
    large = (p0["touched"][order] > 64).astype(np.int64)
    assert max(large[i:i + 64].sum() for i in range(0, len(order), 64)) > 8
    g = gu.run_gpu(sc)
    assert g["K"] == len(b["keys"])
    assert np.array_equal(g["keys"], b["keys"])
    assert np.array_equal(g["values"], b["values"])
    assert np.array_equal(g["ranges"].astype(np.int64), b["ranges"])
    rng = np.random.default_rng(4)
    px, py = rng.integers(0, 1024, 400), rng.integers(0, 768, 400)
    r = composite.composite_pixels(projs[0], px, py, margins=True)
    ok = ~gu.ambiguous(r)
    assert ok.sum() >= 380
    assert np.abs(g["color"][0][:, py, px] - r["color"])[:, ok].max() <= 1e-4


def test_batched_beyond_packed_depth_values():
    """8 views x 2.2M Gaussians = 17.6M (view, Gaussian) entries, past the 2^24
    entries whose depth-sort values carry their pair counts: the batched step (which
    then gathers the counts) renders every view bit for bit like the single-view
    steps (which do not) and lists the same number of pairs."""
    from paper_2503_13086_amd.pipeline import Rasterizer, params_to_device
    sc = scenegen.small_scene(31, 2_200_000, 0, [(96, 64)] * 8, log_scale_mean=-4.5)
    assert len(sc.cams) * sc.n > (1 << 24)
    rz = Rasterizer(0)
    try:
        P = params_to_device(sc.params)
        rz.preprocess(P, sc.n, 0, sc.cams)
        K = rz.bin_sort()
        imgs = [x.clone() for x in rz.image_views(rz.render_fwd())]
        k_single = 0
        for v, c in enumerate(sc.cams):
            rz.preprocess(P, sc.n, 0, [c])
            k_single += rz.bin_sort()
            assert torch.equal(imgs[v], rz.render_fwd().view(3, c["height"], c["width"])), v
    finally:
        rz.close()
    assert K == k_single and K > 0


@pytest.mark.gpu
def test_views_reused_or_changed_between_calls():
    """The device copy of the views is refreshed only when they change: repeating,
    switching and switching back the cameras on one context renders every call bit
    for bit like a fresh context does."""
    from paper_2503_13086_amd.pipeline import Rasterizer, params_to_device
    sc = scenegen.small_scene(41, 3000, 1, [(96, 64), (80, 72)])
    a, b = [sc.cams[0]], [sc.cams[1]]

    def fresh(cams):
        rz = Rasterizer(0)
        try:
            rz.preprocess(params_to_device(sc.params), sc.n, 1, cams)
            rz.bin_sort()
            return rz.render_fwd().clone()
        finally:
            rz.close()

    ref = {"a": fresh(a), "b": fresh(b)}
    rz = Rasterizer(0)
    try:
        P = params_to_device(sc.params)
        for name in ("a", "a", "b", "a", "b", "b"):
            rz.preprocess(P, sc.n, 1, a if name == "a" else b)
            rz.bin_sort()
            assert torch.equal(rz.render_fwd(), ref[name]), name
    finally:
        rz.close()


@pytest.mark.gpu
def test_measurement_probes():
    """The copy probe copies (every byte, including a ragged last workgroup) and the
    FMA probe's chains stay finite, with the flop count its launch shape implies;
    misaligned or odd sizes are refused."""
    import paper_2503_13086_amd as gs
    n = (1 << 20) + 36                     # not a multiple of a workgroup's 256 vectors
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    gs.gs_probe_copy(src, dst, n * 4)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    with pytest.raises(gs.GsError):
        gs.gs_probe_copy(src, dst, n * 4 - 4)
    out = torch.zeros(64 * 256, dtype=torch.float32, device="cuda")
    flops = gs.gs_probe_fma(out, 64, 100)
    torch.cuda.synchronize()
    assert flops == 64 * 256 * 100 * 8 * 2
    assert bool(torch.isfinite(out).all()) and float(out.abs().min()) > 0.0
