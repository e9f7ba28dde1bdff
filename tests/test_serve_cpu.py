"""Scheduling logic of the continuous-batching server, on a fake backend (CPU only).

The fake backend computes probabilities with the oracle and checks, at finalize time, that every
slice of the request was launched, in order, into its own contiguous pool range.
"""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_1908_10070_amd import inputs, serve


class FakeBackend(serve.SliceBackend):
    def __init__(self, U, r, delay_polls=2, fail_on_launch=None):
        self.U, self.r = U, r
        self.written = {}          # pool index -> (modes tuple, lo, hi)
        self.delay = delay_polls
        self.fail_on_launch = fail_on_launch
        self.launches = 0
        self.order = []            # request ids in finalize order
        self.lock = threading.Lock()

    def haf_flops(self, n):
        return float(2 ** (n // 2)) * n ** 3 if n else 0.0

    def launch_step(self, jobs, finished):
        self.launches += 1
        if self.fail_on_launch is not None and self.launches == self.fail_on_launch:
            raise RuntimeError("injected launch failure")
        for modes, lo, hi, idx in jobs:
            assert idx not in self.written or self.written[idx] is None
            self.written[idx] = (tuple(modes.tolist()), lo, hi)
        probs = []
        for r in finished:
            # all slices present, contiguous, in order, covering [0, count)
            cover = []
            for q in range(len(r.slices)):
                rec = self.written.pop(r.pool_off + q)
                assert rec[0] == tuple(r.modes.tolist())
                cover.append((rec[1], rec[2]))
            assert cover == r.slices
            probs.append(oracle.prob_ref(self.U, self.r, r.modes.tolist()))
            self.order.append(r.rid)
        return {"polls": self.delay, "probs": np.array(probs)}

    def done(self, h):
        h["polls"] -= 1
        return h["polls"] <= 0

    def results(self, h):
        return h["probs"]


@pytest.fixture
def setup():
    rng = np.random.default_rng(5)
    m = 8
    U = inputs.haar_unitary(m, rng)
    r = np.full(m, 0.6)
    return U, r, rng


def run_requests(srv, pats):
    futs = [srv.submit(p) for p in pats]
    srv.start()
    out = [f.result(timeout=60) for f in futs]
    srv.stop()
    return out


def test_all_requests_complete_with_oracle_values(setup):
    U, r, rng = setup
    pats = [sorted(rng.choice(8, n, replace=False).tolist()) for n in (0, 2, 4, 6, 8, 4, 2, 8)] + [[1, 1, 3, 3]]
    be = FakeBackend(U, r)
    srv = serve.Server(be, pool_entries=64, max_slice=2, step_flops=50.0, adaptive=False)
    got = run_requests(srv, pats)
    for p, v in zip(pats, got):
        assert v == pytest.approx(oracle.prob_ref(U, r, p), rel=1e-13)
    st = srv.stats()
    assert st["completed"] == len(pats) and st["failed"] == 0 and st["steps"] > 1


def test_admission_waits_for_memory(setup):
    U, r, rng = setup
    # max_slice=1: an n=8 request needs 15 pool entries; the pool holds 20, so at most one such
    # request is admitted at a time, the others wait and are admitted as memory frees.
    pats = [sorted(rng.choice(8, 8, replace=False).tolist()) for _ in range(5)]
    be = FakeBackend(U, r, delay_polls=3)
    srv = serve.Server(be, pool_entries=20, max_slice=1, step_flops=1e9)
    got = run_requests(srv, pats)
    assert len(got) == 5 and srv.max_concurrent == 1
    assert be.order == sorted(be.order)


def test_request_that_can_never_fit_is_rejected(setup):
    U, r, rng = setup
    be = FakeBackend(U, r)
    srv = serve.Server(be, pool_entries=4, max_slice=1)
    f = srv.submit(list(range(8)))  # 15 slices > 4 entries
    with pytest.raises(MemoryError):
        f.result(timeout=1)
    assert srv.stats()["rejected"] == 1


def test_short_requests_are_not_stuck_behind_long_ones(setup):
    U, r, rng = setup
    long = list(range(8))
    shorts = [[0, 1], [2, 3], [4, 5]]
    be = FakeBackend(U, r)
    # small step budget: the long request advances a slice or two per step, the shorts finish early
    srv = serve.Server(be, pool_entries=64, max_slice=1, step_flops=300.0, share=0.5, adaptive=False)
    futs = [srv.submit(long)] + [srv.submit(p) for p in shorts]
    srv.start()
    for f in futs:
        f.result(timeout=30)
    srv.stop()
    assert be.order[-1] == 0  # the long request (rid 0) finished last


def test_injected_launch_failure_fails_only_its_requests(setup):
    U, r, rng = setup
    pats = [[0, 1], [2, 3], [4, 5], [6, 7], [0, 2]]
    be = FakeBackend(U, r, fail_on_launch=2)
    srv = serve.Server(be, pool_entries=64, max_slice=4096, step_flops=1.0, share=0.01, inflight=1,
                       adaptive=False)
    futs = [srv.submit(p) for p in pats]
    srv.start()
    outcomes = []
    for f in futs:
        try:
            outcomes.append(f.result(timeout=30))
        except RuntimeError:
            outcomes.append("failed")
    srv.stop()
    assert outcomes.count("failed") >= 1
    assert any(o != "failed" for o in outcomes[2:])  # serving continued after the failure
    assert srv.stats()["failed"] == outcomes.count("failed")


def test_slice_plan_depends_only_on_n():
    assert serve.slice_plan(0) == [] and serve.slice_plan(5) == []
    assert serve.slice_plan(8) == [(0, 15)]
    s = serve.slice_plan(32, 4096)
    assert s[0] == (0, 4096) and s[-1][1] == 2 ** 16 - 1 and len(s) == 16
    assert all(a[1] == b[0] for a, b in zip(s, s[1:]))


def test_oldest_request_draws_from_the_budget_after_its_free_slice(setup):
    """The oldest request gets one slice outside the step budget and then competes for the rest like
    the others (it is not capped at one slice per step when budget is left)."""
    U, r, rng = setup
    long = list(range(8))  # 15 slices of one subset each
    be = FakeBackend(U, r)
    srv = serve.Server(be, pool_entries=64, max_slice=1, step_flops=1e9, share=1.0)
    srv.submit(long)
    srv.submit([0, 1])
    srv._admit()
    jobs, finished = srv._build_step()
    assert len(jobs) == 16 and len(finished) == 2


def test_adaptive_budget_grows_with_backlog(setup):
    """With the adaptive budget a step takes at least the backlog over the steps in flight: a queue of
    40 one-slice requests at a tiny fixed budget goes in a few steps instead of two requests per step."""
    U, r, rng = setup
    pats = [sorted(rng.choice(8, 4, replace=False).tolist()) for _ in range(40)]
    steps = {}
    for adaptive in (False, True):
        be = FakeBackend(U, r)
        srv = serve.Server(be, pool_entries=256, max_slice=4096, step_flops=1.0, share=1.0, inflight=2,
                           adaptive=adaptive)
        out = run_requests(srv, pats)
        assert np.allclose(out, [oracle.prob_ref(U, r, p) for p in pats], rtol=1e-12)
        steps[adaptive] = srv.stats()["steps"]
    assert steps[False] >= 20 and steps[True] <= 8, steps  # fixed: one request plus the oldest per step
