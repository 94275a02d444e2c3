"""Serving loop (continuous batching over a resident, growing field) through the
C ABI: each job's per-iteration results are the same alone and in the mix, every
job runs its T_I planned iterations, the field grows with its Adam state intact,
and admission keeps the footprint within the HBM budget."""
import numpy as np
import pytest
import torch

import scenegen

pytestmark = pytest.mark.gpu


def _stream(n_arr=6, seed=11, size=(96, 64)):
    return scenegen.serving_stream(seed=seed, n_arrivals=n_arr, n0=3000, add=(400, 900), size=size,
                                   mean_interarrival=0.05)


def _engine(st, **kw):
    from paper_2503_13086_amd.serving import Engine, Field
    fld = Field(st.initial, st.sh_degree, capacity=kw.pop("capacity", 0))
    return Engine(fld, **kw)


def _targets(st):
    return [torch.as_tensor(a.target()).reshape(-1).cuda() for a in st.arrivals]


def test_field_growth_keeps_state():
    from paper_2503_13086_amd.serving import Field
    st = _stream(4)
    f = Field(st.initial, st.sh_degree, capacity=3000)
    f.m[:, : f.n].fill_(0.5)
    f.step[: f.n].fill_(3)
    ref = [st.initial]
    for a in st.arrivals:
        f.append(a.block)
        ref.append(a.block)
    ref = np.concatenate(ref, axis=1)
    assert f.n == ref.shape[1] and f.growths >= 2 and f.cap >= f.n
    assert np.array_equal(f.params[:, : f.n].cpu().numpy(), ref)
    n0 = st.initial.shape[1]
    assert (f.m[:, :n0] == 0.5).all() and (f.m[:, n0: f.n] == 0).all()
    assert (f.step[:n0] == 3).all() and (f.step[n0: f.n] == 0).all()


def test_alone_equals_mix():
    """One engine step over three jobs' views against three single-job steps from
    the same field snapshot: images and losses bit for bit, gradient = sum of the
    single-view gradients within fp32 atomics."""
    st = _stream(3)
    eng = _engine(st, max_slots=4, t_i=8, w_l1=0.47, w_dssim=0.12, w_load=0.41)    # Eq. 10 weights
    tg = _targets(st)
    try:
        jobs = [eng.register(a.cam, tg[i], a.overlap, a.block) for i, a in enumerate(st.arrivals)]
        snap = eng.field.snapshot()
        trained = list(eng.trained)
        nexts = [j.next for j in jobs]
        mix = eng.step(jobs, record=True)
        alone = []
        for j in jobs:
            eng.field.restore(snap)
            eng.trained[:] = trained
            for jj, nx in zip(jobs, nexts):
                jj.next = nx
            alone.append(eng.step([j], record=True))
    finally:
        eng.close()
    gsum = torch.zeros_like(mix["grad"])
    for k, a in enumerate(alone):
        assert a["views"] == [mix["views"][k]]
        assert torch.equal(a["color"][0], mix["color"][k])
        assert a["loss"][0].item() == mix["loss"][k].item()
        gsum += a["grad"]
    g = mix["grad"]
    assert (g - gsum).abs().max().item() <= 1e-5 * g.abs().max().item()


def test_serving_runs_every_planned_iteration():
    st = _stream(6)
    eng = _engine(st, max_slots=4, t_i=10, capacity=3000)
    try:
        stats = eng.run(st.arrivals, _targets(st), time_scale=0.0)
        trained = list(eng.trained)
        n = eng.field.n
    finally:
        eng.close()
    assert stats.iterations == 6 * 10 and sum(trained) == 60
    assert len(stats.latencies) == 6 and min(stats.latencies) > 0
    assert stats.max_batch > 1                     # arrivals at once are batched
    assert n == st.initial.shape[1] + sum(a.block.shape[1] for a in st.arrivals)
    assert stats.field_growths >= 1


def test_plain_loop_is_one_view_per_step():
    st = _stream(3)
    eng = _engine(st, max_slots=1, t_i=6)
    try:
        stats = eng.run(st.arrivals, _targets(st), time_scale=0.0)
    finally:
        eng.close()
    assert stats.max_batch == 1 and stats.steps == 18 and len(stats.latencies) == 3


def test_admission_respects_hbm_budget():
    """A budget with room for about two jobs' working sets: no step ever runs more
    than the budget allows and the measured footprint stays within it."""
    st = _stream(5)
    n_final = st.initial.shape[1] + sum(a.block.shape[1] for a in st.arrivals)
    eng = _engine(st, max_slots=8, t_i=6, capacity=n_final)
    try:
        px = st.arrivals[0].cam["width"] * st.arrivals[0].cam["height"]
        resident = eng.field.bytes_at(n_final) + 5 * 12 * px
        # the smallest per-view working set the engine can estimate (no pairs, the
        # initial field): at most two views ever fit
        eng.pairs_per_view = 0
        per_view = eng._view_bytes(st.initial.shape[1], px)
        eng.budget = resident + int(2.5 * per_view) + 2 * 12 * px * 2
        stats = eng.run(st.arrivals, _targets(st), time_scale=0.0)
    finally:
        eng.close()
    assert len(stats.latencies) == 5
    assert 1 <= stats.max_batch <= 2
    assert stats.peak_bytes <= eng.budget


@pytest.mark.parametrize("slots", [1, 3])
def test_checkpoint_resume_ends_with_the_same_bits(tmp_path, slots):
    """With the ordered backward (gradients the same bits on every run), the plain
    loop and continuous batching: a run stopped with jobs in flight (after 18
    steps of one view, or 6 steps of three), saved, loaded into a fresh engine and resumed ends with the same
    parameters, moments, step counters and per-image training counts, bit for bit,
    as an uninterrupted run."""
    import paper_2503_13086_amd as gs
    from paper_2503_13086_amd.serving import Engine
    st = _stream(3)
    tg = _targets(st)
    kw = dict(max_slots=slots, t_i=12, seed=2, w_l1=0.47, w_dssim=0.12, w_load=0.41)
    ref = _engine(st, **kw)
    try:
        gs.gs_set_backward_order(ref.rz.ctx, gs.GS_BWD_ORDERED)
        ref.run(st.arrivals, tg, time_scale=0.0)
        want = {k: getattr(ref.field, k)[..., : ref.field.n].cpu().numpy().copy() for k in ("params", "m", "v", "step")}
        want_trained = list(ref.trained)
    finally:
        ref.close()
    eng = _engine(st, **kw)
    path = str(tmp_path / "serve.safetensors")
    try:
        gs.gs_set_backward_order(eng.rz.ctx, gs.GS_BWD_ORDERED)
        eng.run(st.arrivals, tg, time_scale=0.0, max_steps=18 if slots == 1 else 6)
        assert any(not j.finished for j in eng.jobs) and (slots > 1 or len(eng.cams) < 3)
        eng.save(path)
    finally:
        eng.close()
    back = Engine.load(path)
    try:
        gs.gs_set_backward_order(back.rz.ctx, gs.GS_BWD_ORDERED)
        back.run(st.arrivals, tg, time_scale=0.0)
        assert back.trained == want_trained
        for k, v in want.items():
            got = getattr(back.field, k)[..., : back.field.n].cpu().numpy()
            assert got.shape == v.shape and np.array_equal(got.view(np.uint32), v.view(np.uint32)), k
    finally:
        back.close()
