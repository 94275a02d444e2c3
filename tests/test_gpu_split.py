"""Binning of scenes with large splats, through the C ABI: waves of 64 entries
with more than 2048 candidate tiles hand their largest entries to the chunk
passes of the count and the emission.  The listed pairs,
their order and the tile ranges must equal the oracle's bit for bit, with the
split lists fitting (every large entry of a heavy wave split), with the
emission's entry list full (the entries past it stay with their waves), with
both lists full (tile edge 8), in rect mode (emission only) and in exact mode
(outcomes read from the exact pass's store)."""
import numpy as np
import pytest

import scenegen
import oracle
import paper_2503_13086_amd as gs
from paper_2503_13086_amd.pipeline import Rasterizer, params_to_device
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

SPLIT_WAVE, CHUNK, LISTS = 2048, 512, 64   # the split rule of the binning kernels


def _scene(log_scale_mean, sizes=((320, 240), (200, 150))):
    return scenegen.small_scene(201, 3000, 1, list(sizes), log_scale_mean=log_scale_mean)


def _threshold(c):
    """The largest t (64 doubled up to 8192) leaving at most SPLIT_WAVE candidates
    to the entries of at most t (64 if none does)."""
    for t in (8192, 4096, 2048, 1024, 512, 256, 128):
        if c[c <= t].sum() <= SPLIT_WAVE:
            return t
    return 64


def _split_work(projs, order_by_depth):
    """Per list: entries a heavy wave splits and their chunk items, from the
    oracle's rects (index order, or the depth order of the emission); wave w
    uses list w % LISTS."""
    cand = np.concatenate([np.where(p["visible"], (p["tx1"] - p["tx0"] + 1) * (p["ty1"] - p["ty0"] + 1), 0)
                           for p in projs]).astype(np.int64)
    if order_by_depth:
        depth = np.concatenate([np.where(p["visible"], p["depth_bits"], 0xffffffff) for p in projs])
        cand = cand[np.argsort(depth.astype(np.uint64), kind="stable")]
    ents, items = np.zeros(LISTS, np.int64), np.zeros(LISTS, np.int64)
    for w0 in range(0, len(cand), 64):
        c = cand[w0:w0 + 64]
        if c.sum() > SPLIT_WAVE:
            big = c[c > _threshold(c)]
            ents[(w0 // 64) % LISTS] += len(big)
            items[(w0 // 64) % LISTS] += int(((big + CHUNK - 1) // CHUNK).sum())
    return ents, items


CASES = {
    # (log-scale mean, tile edge, view sizes): what the lists hold
    "fits": (-2.2, 16, ((320, 240), (200, 150))),
    "emit_entries_full": (-1.6, 16, ((320, 240), (200, 150))),
    "both_full_tile8": (-1.6, 8, ((640, 480), (400, 300))),
}


@pytest.mark.parametrize("case", list(CASES))
def test_split_binning_bit_exact(case):
    ls, tile, sizes = CASES[case]
    sc = _scene(ls, sizes)
    projs = oracle.project_views(sc.params, sc.n, sc.sh_degree, sc.cams, tile)
    NV = len(sc.cams) * sc.n
    icap = NV // (16 * LISTS) + 256   # slots per list
    ecap = NV // (64 * LISTS) + 64
    c_ents, c_items = _split_work(projs, False)
    e_ents, e_items = _split_work(projs, True)
    assert c_ents.sum() > 0 and e_ents.sum() > 0, "the scene must split work"
    if case == "fits":
        assert c_items.max() <= icap and e_ents.max() <= ecap and e_items.max() <= icap
    elif case == "emit_entries_full":
        assert c_items.max() <= icap and e_ents.max() > ecap
    else:
        assert c_items.max() > icap and e_ents.max() > ecap
    b = oracle.bin_pairs(projs, sc.cams, tile, cull="ellipse")
    print(f"[split] {case}: K={len(b['keys'])}, count items per list <= {c_items.max()}/{icap}, emission "
          f"entries per list <= {e_ents.max()}/{ecap}", flush=True)
    g = gu.run_gpu(sc, tile=tile)
    print(f"[split] {case}: binned again after a capacity report: {g['retried']}", flush=True)
    assert g["K"] == len(b["keys"])
    keys, values, views = gu.valid_pairs(g)
    assert np.array_equal(keys, b["keys"])
    assert np.array_equal(values, b["values"])
    assert np.array_equal(views, b["views"].astype(np.uint32))
    assert np.array_equal(g["ranges"].astype(np.int64), b["ranges"])


def test_split_binning_rect_mode_bit_exact():
    sc = _scene(-2.2)
    projs = oracle.project_views(sc.params, sc.n, sc.sh_degree, sc.cams, 16)
    b = oracle.bin_pairs(projs, sc.cams, 16, cull="rect")
    g = gu.run_gpu(sc, cull="rect")
    assert g["K"] == len(b["keys"])
    assert np.array_equal(g["keys"], b["keys"])
    assert np.array_equal(g["values"], b["values"])
    assert np.array_equal(g["ranges"].astype(np.int64), b["ranges"])


def test_split_binning_exact_mode_bit_exact():
    """Exact mode: every large entry's outcomes come from the exact pass's store
    (grown after the first binning reports it too small)."""
    sc = _scene(-2.2)
    projs = oracle.project_views(sc.params, sc.n, sc.sh_degree, sc.cams, 16)
    b = oracle.bin_pairs(projs, sc.cams, 16, cull="ellipse")
    rz = Rasterizer(0)
    try:
        gs.gs_set_cull(rz.ctx, gs.GS_CULL_ELLIPSE_EXACT)
        P = params_to_device(sc.params)
        for attempt in range(2):
            rz.preprocess(P, sc.n, sc.sh_degree, sc.cams)
            K = rz.bin_sort()
            try:
                rz.sync_status()
                break
            except gs.GsError as e:
                assert attempt == 0 and e.status == gs.GS_ERR_CAPACITY
        assert K == len(b["keys"])
        keys = rz.buffer(gs.GS_BUF_KEYS).cpu().numpy().view(np.uint64)
        values = rz.buffer(gs.GS_BUF_VALUES).cpu().numpy().view(np.uint32)
        ranges = rz.buffer(gs.GS_BUF_RANGES).cpu().numpy().view(np.uint32).reshape(-1, 2)
        assert np.array_equal(keys, b["keys"])
        assert np.array_equal(values, b["values"])
        assert np.array_equal(ranges.astype(np.int64), b["ranges"])
    finally:
        rz.close()
