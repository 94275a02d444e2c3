"""Device-side status of the binning, through the C ABI: a binning that does not
wait for its pair count, pair buffers forced too small (the kernels do nothing,
gs_sync_status reports GS_ERR_CAPACITY with the size needed, the fused backward
+ Adam leaves every buffer untouched, the next binning grows and matches a fresh
run), the store of exact cutoff outcomes forced to overflow the same way, and the
exact cull mode (every cutoff test in FP64) listing the same pairs as the default
fp32-first mode and the oracle."""
import numpy as np
import pytest
import torch

import scenegen
import oracle
import paper_2503_13086_amd as gs
from paper_2503_13086_amd.pipeline import Rasterizer, params_to_device
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _scene():
    return scenegen.small_scene(101, 2000, 3, [(100, 75), (64, 48)], log_scale_mean=-2.8, bg=(0.1, 0.2, 0.3))


def _step(rz, P, sc, m, v, step, count):
    rz.preprocess(P, sc.n, sc.sh_degree, sc.cams)
    K = rz.bin_sort(count=count)
    color = rz.render_fwd()
    tgt = rz.pack_images(sc.targets)
    _, dl = rz.loss(color, tgt, 0.8, 0.2)
    rz.render_bwd_adam(dl, m, v, step, view_lr_scale=[1.0, 0.5])
    return K, color


def test_binning_without_waiting_matches_waiting():
    sc = _scene()
    outs = []
    for count in (True, False):
        rz = Rasterizer(0)
        try:
            P = params_to_device(sc.params)
            rz.preprocess(P, sc.n, sc.sh_degree, sc.cams)
            rz.bin_sort(count=True)            # first binning sizes the buffers
            rz.preprocess(P, sc.n, sc.sh_degree, sc.cams)
            K = rz.bin_sort(count=count)
            color = rz.render_fwd()
            rz.sync_status()
            keys = rz.buffer(gs.GS_BUF_KEYS).cpu().numpy()
            outs.append((K, color.cpu().numpy(), keys))
        finally:
            rz.close()
    assert outs[1][0] is None and outs[0][0] == len(outs[1][2])
    assert np.array_equal(outs[0][2], outs[1][2])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_pair_capacity_overflow_is_reported_and_recovered():
    sc = _scene()
    rz = Rasterizer(0)
    try:
        P = params_to_device(sc.params)
        rz.preprocess(P, sc.n, sc.sh_degree, sc.cams)
        K = rz.bin_sort(count=True)
        ref_keys = rz.buffer(gs.GS_BUF_KEYS).cpu().numpy()
        ref_color = rz.render_fwd().cpu().numpy()
        torch.cuda.synchronize()
        gs.gs_reserve_pairs(rz.ctx, K // 2)
        m, v = torch.zeros_like(P), torch.zeros_like(P)
        step = torch.zeros(sc.n, dtype=torch.int32, device=P.device)
        before = [x.clone() for x in (P, m, v, step)]
        print(f"[status] overflow step: K={K}, capacity {K // 2}", flush=True)
        _step(rz, P, sc, m, v, step, count=False)
        with pytest.raises(gs.GsError) as ei:
            rz.sync_status()
        assert ei.value.status == gs.GS_ERR_CAPACITY
        assert f"{K} pairs needed" in str(ei.value)
        for a, b in zip(before, (P, m, v, step)):
            assert torch.equal(a, b), "a failed step must leave parameters, moments and steps untouched"
        # the next binning grows to the size reported and matches the reference
        print("[status] recovery step", flush=True)
        _, color = _step(rz, P, sc, m, v, step, count=False)
        rz.sync_status()
        assert int(step.min()) == 1
        torch.cuda.synchronize()
        assert np.array_equal(color.cpu().numpy(), ref_color)
        rz.preprocess(before[0], sc.n, sc.sh_degree, sc.cams)
        rz.bin_sort(count=False)
        rz.sync_status()
        assert np.array_equal(rz.buffer(gs.GS_BUF_KEYS).cpu().numpy(), ref_keys)
    finally:
        rz.close()


@pytest.mark.parametrize("name", ["ragged2v_sh3", "c1_10k_sh0", "ragged3v_sh1", "sh2_dense"])
def test_exact_mode_lists_equal_fp32_first_mode(name):
    from tests.test_gpu_parity import SCENES
    sc = SCENES[name]()
    projs = oracle.project_views(sc.params, sc.n, sc.sh_degree, sc.cams)
    b = oracle.bin_pairs(projs, sc.cams, 16, cull="ellipse")
    print(f"[status] exact mode {name}", flush=True)
    ge = gu.run_gpu(sc, cull="exact")
    gf = gu.run_gpu(sc, cull="ellipse")
    for g in (ge, gf):
        assert g["K"] == len(b["keys"])
        assert np.array_equal(g["keys"], b["keys"])
        assert np.array_equal(g["values"], b["values"])
        assert np.array_equal(g["ranges"].astype(np.int64), b["ranges"])
    assert np.array_equal(ge["color"][0], gf["color"][0])


def test_exact_outcome_store_overflow_is_reported_and_recovered():
    """Large splats (rects of several hundred tiles) in exact mode need more outcome
    words than a fresh context holds: the first binning reports GS_ERR_CAPACITY,
    the second fits and lists the oracle's pairs."""
    sc = scenegen.small_scene(77, 300, 0, [(320, 320)], log_scale_mean=-0.7)
    projs = oracle.project_views(sc.params, sc.n, sc.sh_degree, sc.cams)
    b = oracle.bin_pairs(projs, sc.cams, 16, cull="ellipse")
    big = (projs[0]["touched"] > 64).sum()
    words = int(((projs[0]["touched"][projs[0]["touched"] > 64] + 31) // 32).sum())
    print(f"[status] exact store: {big} splats of > 64 tiles, {words} words", flush=True)
    assert words > sc.n // 64 + 1024
    rz = Rasterizer(0)
    try:
        gs.gs_set_cull(rz.ctx, gs.GS_CULL_ELLIPSE_EXACT)
        P = params_to_device(sc.params)
        rz.preprocess(P, sc.n, sc.sh_degree, sc.cams)
        rz.bin_sort(count=True)
        with pytest.raises(gs.GsError) as ei:
            rz.sync_status()
        assert ei.value.status == gs.GS_ERR_CAPACITY
        rz.preprocess(P, sc.n, sc.sh_degree, sc.cams)
        K = rz.bin_sort(count=True)
        rz.sync_status()
        assert K == len(b["keys"])
        assert np.array_equal(rz.buffer(gs.GS_BUF_KEYS).cpu().numpy().view(np.uint64), b["keys"])
        assert np.array_equal(rz.buffer(gs.GS_BUF_RANGES).cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64),
                              b["ranges"])
    finally:
        rz.close()


@pytest.mark.parametrize("cap", [None, 3, 12_000_000])
def test_binning_into_large_capacity_matches(cap):
    """Pair buffers much larger than K (a multiple of K, and 12M pairs: a digit
    table of more than 2048 blocks, so the capacity's chunking differs from the
    count's): binning without waiting sorts exactly K pairs, as a counted binning does."""
    sc = _scene()
    rz = Rasterizer(0)
    try:
        P = params_to_device(sc.params)
        rz.preprocess(P, sc.n, sc.sh_degree, sc.cams)
        K = rz.bin_sort(count=True)
        ref_keys = rz.buffer(gs.GS_BUF_KEYS).cpu().numpy()
        ref_ranges = rz.buffer(gs.GS_BUF_RANGES).cpu().numpy()
        ref_color = rz.render_fwd().cpu().numpy()
        if cap is not None:
            gs.gs_reserve_pairs(rz.ctx, cap * K if cap < 100 else cap)
        print(f"[status] K={K}, capacity {cap}", flush=True)
        for _ in range(2):
            rz.preprocess(P, sc.n, sc.sh_degree, sc.cams)
            assert rz.bin_sort(count=False) is None
            color = rz.render_fwd()
            rz.sync_status()
            assert np.array_equal(rz.buffer(gs.GS_BUF_KEYS).cpu().numpy(), ref_keys)
            assert np.array_equal(rz.buffer(gs.GS_BUF_RANGES).cpu().numpy(), ref_ranges)
            assert np.array_equal(color.cpu().numpy(), ref_color)
    finally:
        rz.close()
