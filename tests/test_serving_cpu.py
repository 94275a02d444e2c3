"""Host logic of the serving loop on the CPU: a stand-in rasterizer records the
calls, so admission, batching, per-job iteration plans, Eq. 6-8 rates handed to
the optimizer and latency accounting are checked without a GPU."""
import numpy as np
import pytest
import torch

import scenegen
from oracle import schedule
from paper_2503_13086_amd.serving import Engine, Field


class FakeRasterizer:
    def __init__(self, bytes_per_view=0):
        self.calls = []
        self.bytes_per_view = bytes_per_view
        self.held = 0
        self.ctx = object()

    def set_views(self, cams, tile=16):
        self.cams = list(cams)
        self.P = sum(c["width"] * c["height"] for c in cams)

    def preprocess(self, params, n, sh_degree, cams=None, stream=None):
        self.n = n
        self.held = max(self.held, self.bytes_per_view * len(self.cams))

    def bin_sort(self, stream=None):
        return 5 * self.n * len(self.cams)

    def render_fwd(self, color=None, stream=None):
        color.fill_(0.5)
        return color

    def loss(self, color, target, w_l1=1.0, w_dssim=0.0, loss_out=None, dL_dcolor=None, stream=None):
        loss_out.fill_(1.0)
        dL_dcolor.fill_(0.0)
        return loss_out, dL_dcolor

    def render_bwd(self, dL_dcolor, grad=None, accumulate=False, stream=None):
        grad[:, : self.n].fill_(1.0)
        return grad

    def adam_step(self, grad, m, v, step, lr_group, view_lr_scale=None, group_mask=1, **kw):
        self.calls.append(("adam", list(view_lr_scale), [id(c) for c in self.cams]))

    def render_bwd_adam(self, dL_dcolor, m, v, step, lr_group, view_lr_scale=None, group_mask=1, **kw):
        self.calls.append(("adam", list(view_lr_scale), [id(c) for c in self.cams]))

    def image_views(self, flat):
        out, a = [], 0
        for c in self.cams:
            b = a + 3 * c["width"] * c["height"]
            out.append(flat[a:b].view(3, c["height"], c["width"]))
            a = b
        return out

    def memory_bytes(self):
        return self.held

    def close(self):
        pass


def _stream(n_arr=7, seed=3):
    return scenegen.serving_stream(seed=seed, n_arrivals=n_arr, n0=500, add=(50, 120), size=(32, 24),
                                   mean_interarrival=0.01, n_landmarks=4000)


def _targets(st):
    return [torch.as_tensor(a.target()).reshape(-1) for a in st.arrivals]


def _engine(st, **kw):
    fld = Field(st.initial, st.sh_degree, device="cpu", capacity=kw.pop("capacity", 0))
    rz = FakeRasterizer(kw.pop("bytes_per_view", 0))
    return Engine(fld, rasterizer=rz, **kw), rz


def test_every_job_runs_its_plan_and_batches_fill():
    st = _stream(7)
    eng, rz = _engine(st, max_slots=3, t_i=12)
    stats = eng.run(st.arrivals, _targets(st), time_scale=0.0)
    assert stats.iterations == 7 * 12 and sum(eng.trained) == 7 * 12
    assert stats.max_batch == 3 and len(stats.latencies) == 7
    assert eng.field.n == 500 + sum(a.block.shape[1] for a in st.arrivals)
    # per image: the number of iterations it was trained equals the plans' counts
    counts = np.zeros(7, np.int64)
    for j in eng.jobs:
        for v in j.plan:
            counts[v] += 1
    assert counts.tolist() == eng.trained


def test_plain_loop_serves_in_arrival_order():
    st = _stream(4)
    eng, rz = _engine(st, max_slots=1, t_i=5)
    stats = eng.run(st.arrivals, _targets(st), time_scale=0.0)
    assert stats.steps == 20 and stats.max_batch == 1
    # all arrive at once: completions in arrival order, each later job waited for the earlier ones
    assert [j.image for j in eng.jobs] == [0, 1, 2, 3]
    assert (np.diff(stats.latencies) > 0).all()


def test_rates_given_to_adam_follow_eq6_to_eq8():
    """Each view's scale is its Eq. 8 rate (trained counts before the step, T_a
    = 200) over the group base rate, as the oracle's schedule computes it."""
    st = _stream(4)
    eng, rz = _engine(st, max_slots=4, t_i=6)
    tg = _targets(st)
    jobs = [eng.register(a.cam, tg[i], a.overlap, a.block) for i, a in enumerate(st.arrivals)]
    for _ in range(3):
        trained = list(eng.trained)
        views = [j.plan[j.next] for j in jobs]
        eng.step(jobs)
        scales = rz.calls[-1][1]
        M = eng.M.copy()
        np.fill_diagonal(M, 0.0)
        cur = [schedule.lr_current(t, 1.6e-4, 1.6e-6, 200.0) for t in trained]
        for v, s in zip(views, scales):
            assert s == pytest.approx(schedule.lr_neighbourhood(v, cur, M) / 1.6e-4, rel=1e-14)
        for v in views:
            trained[v] += 1
        assert eng.trained == trained


def test_plans_follow_the_schedule():
    st = _stream(5)
    eng, rz = _engine(st, max_slots=2, t_i=20, seed=9)
    tg = _targets(st)
    rng = np.random.default_rng(9)
    for i, a in enumerate(st.arrivals):
        job = eng.register(a.cam, tg[i], a.overlap, a.block)
        w = schedule.hierarchical_weights(eng.M, i)
        assert job.plan == schedule.iteration_plan(w, i + 1, 10, 20, rng.random(i + 1))


def test_admission_waits_for_memory():
    """With room for two views' working sets, never more than two jobs run at once
    even with free slots, and every job still completes."""
    st = _stream(5)
    n_final = 500 + sum(a.block.shape[1] for a in st.arrivals)
    eng, rz = _engine(st, max_slots=8, t_i=4, bytes_per_view=10_000, capacity=n_final)
    px = 32 * 24
    eng.pairs_per_view = 0
    per_view = eng._view_bytes(500, px)            # smallest field: at most two views ever fit
    eng.budget = eng.field.bytes_at(n_final) + 5 * 12 * px + int(2.5 * per_view) + 2 * 12 * px * 2
    stats = eng.run(st.arrivals, _targets(st), time_scale=0.0)
    assert len(stats.latencies) == 5 and stats.max_batch == 2
    assert stats.peak_bytes <= eng.budget


def test_budget_too_small_raises():
    st = _stream(2)
    eng, rz = _engine(st, max_slots=2, t_i=2, hbm_budget=1000)
    with pytest.raises(MemoryError):
        eng.run(st.arrivals, _targets(st), time_scale=0.0)


def test_checkpoint_round_trip_and_resume(tmp_path):
    """Engine.save / Engine.load restore the field (parameters, moments, step
    counters, capacity), images, overlap matrix, trained counts, jobs and the
    planning generator exactly; a run stopped after 7 steps, saved, loaded and
    resumed serves the same plans, the same number of steps and the same
    per-image training counts as an uninterrupted run."""
    st = _stream(5)
    ref, _ = _engine(st, max_slots=2, t_i=9, seed=4)
    ref_stats = ref.run(st.arrivals, _targets(st), time_scale=0.0)

    eng, _ = _engine(st, max_slots=2, t_i=9, seed=4)
    eng.run(st.arrivals, _targets(st), time_scale=0.0, max_steps=7)
    assert eng.stats.steps == 7 and any(not j.finished for j in eng.jobs)
    g = torch.Generator().manual_seed(0)
    n = eng.field.n
    for k in ("m", "v"):
        getattr(eng.field, k)[:, :n] = torch.rand(eng.field.n_p, n, generator=g)
    eng.field.step[:n] = torch.randint(0, 100, (n,), generator=g, dtype=torch.int32)
    path = str(tmp_path / "engine.safetensors")
    eng.save(path)
    back = Engine.load(path, device="cpu", rasterizer=FakeRasterizer())
    for k in ("params", "m", "v", "step"):
        assert torch.equal(getattr(back.field, k)[..., :n], getattr(eng.field, k)[..., :n]), k
    assert back.field.n == n and back.field.cap == eng.field.cap
    assert np.array_equal(back.M, eng.M) and back.trained == eng.trained
    assert [(j.image, j.plan, j.next) for j in back.jobs] == [(j.image, j.plan, j.next) for j in eng.jobs]
    assert all(torch.equal(a, b) for a, b in zip(back.targets, eng.targets))
    for ca, cb in zip(back.cams, eng.cams):
        assert set(ca) == set(cb) and all(np.array_equal(np.asarray(ca[k]), np.asarray(cb[k])) for k in ca)
    assert back.elapsed == eng.elapsed and back.stats.steps == 7

    stats = back.run(st.arrivals, _targets(st), time_scale=0.0)
    assert stats.steps == ref_stats.steps and stats.iterations == ref_stats.iterations
    assert back.trained == ref.trained
    assert [j.plan for j in back.jobs] == [j.plan for j in ref.jobs]
    assert len(stats.latencies) == 5
