"""The library's host-side schedule (gs_sched_weights, gs_sched_plan, gs_sched_lr;
Sec. IV-C Eq. 3-5, Sec. IV-D Eq. 6-8) against the oracle's schedule, bit for bit,
on random overlap graphs.  Host-only entry points: runs without a GPU."""
import numpy as np
import pytest

import paper_2503_13086_amd as gs
from oracle import schedule


def _graph(rng, n, density):
    A = (rng.random((n, n)) < density) * rng.random((n, n))
    A = np.maximum(A, A.T)
    np.fill_diagonal(A, rng.random(n))        # the diagonal is ignored by both sides
    return A


@pytest.mark.parametrize("n,density,seed", [(1, 0.0, 0), (2, 1.0, 1), (7, 0.3, 2), (40, 0.05, 3),
                                            (150, 0.02, 4), (200, 0.5, 5)])
def test_weights_plan_lr_match_oracle(n, density, seed):
    rng = np.random.default_rng(seed)
    A = _graph(rng, n, density)
    new = int(rng.integers(0, n))
    w, lay = gs.gs_sched_weights(A, new)
    ref = schedule.hierarchical_weights(A, new)
    expect = np.full(n, -1.0)
    for i, x in ref.items():
        expect[i] = x
    assert np.array_equal(w, expect)
    assert lay[new] == 1 and ((lay == 0) == (w < 0)).all()
    for t_i in (200, 7, 1, 0):
        u = rng.random(n)
        plan, share = gs.gs_sched_plan(w, 10, t_i, u)
        assert plan.tolist() == schedule.iteration_plan(ref, n, 10, t_i, u)
        ob = schedule.local_budget(ref, 10, t_i)
        assert {i: int(share[i]) for i in ob} == ob and share[[i for i in range(n) if i not in ob]].sum() == 0
    trained = rng.integers(0, 450, n)
    cur, lr = gs.gs_sched_lr(trained, A, 1.6e-4, 1.6e-6, 200.0)
    for j in range(n):
        assert cur[j] == schedule.lr_current(int(trained[j]), 1.6e-4, 1.6e-6, 200.0)
        Mz = A.copy()
        np.fill_diagonal(Mz, 0.0)
        assert lr[j] == schedule.lr_neighbourhood(j, list(cur), Mz)


def test_sched_argument_checks():
    A = np.zeros((3, 3))
    with pytest.raises(gs.GsError):
        gs.gs_sched_weights(A, 3)
    A[0, 1] = -0.1
    with pytest.raises(gs.GsError):
        gs.gs_sched_weights(A, 0)
    A[0, 1] = np.nan
    with pytest.raises(gs.GsError):
        gs.gs_sched_lr([0, 0, 0], A, 1e-4, 1e-6, 200.0)
    with pytest.raises(gs.GsError):
        gs.gs_sched_lr([0, -1, 0], np.zeros((3, 3)), 1e-4, 1e-6, 200.0)
    with pytest.raises(gs.GsError):
        gs.gs_sched_plan([1.0, 0.5, -1.0], 0, 10, [0.1, 0.2, 0.3])
