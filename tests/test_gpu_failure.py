"""Failure detection through the C ABI on the GPU: the launch-failure hook (gbs_debug_fault_inject /
GBS_FAULT_INJECT) fails exactly one call, enqueues nothing and leaves the context usable; a server
fails only the requests that the failed launch carried and keeps serving; the debug symmetry check
rejects an asymmetric caller matrix. The injected failure is raised on the host before any kernel is
enqueued, so no kernel ever runs in a failed state."""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

import oracle
from paper_1908_10070_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_10070_amd import gbs
    yield gbs, torch.device("cuda", 0)
    gbs.debug_fault_inject(0)
    gbs.debug_check_symmetry(False)


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def test_injected_failure_fails_one_call(env):
    gbs, dev = env
    ctx = gbs.Context(0)
    A_host = inputs.random_symmetric(12, 16, np.random.default_rng(8100))
    A = to_dev(A_host, dev)
    ref = ctx.haf_batch(A).cpu().numpy()
    out = to_dev(np.zeros(16, np.complex128), dev)
    try:
        gbs.debug_fault_inject(3)
        ctx.haf_batch(A, out=out)
        ctx.haf_batch(A, out=out)
        out.zero_()
        with pytest.raises(gbs.GBSError) as ei:
            ctx.haf_batch(A, out=out)
        assert ei.value.status == gbs.GBS_EHIP and "injected" in str(ei.value)
        assert not out.cpu().numpy().any()  # nothing was enqueued
        # the fourth and later calls run normally
        assert np.array_equal(ctx.haf_batch(A).cpu().numpy(), ref)
        assert np.max(np.abs(ref - oracle.haf_enum_batch(A_host)) / np.abs(ref)) < 1e-9
    finally:
        gbs.debug_fault_inject(0)


def test_fault_inject_from_environment(env):
    """GBS_FAULT_INJECT=launch:2 in the environment: the second compute call of the process fails."""
    code = textwrap.dedent("""
        import numpy as np, torch
        from paper_1908_10070_amd import gbs
        ctx = gbs.Context(0)
        A = torch.ones((2, 8, 8), dtype=torch.complex128, device="cuda")
        h = ctx.haf_batch(A).cpu().numpy()
        assert np.allclose(h, 105, rtol=1e-12), h
        try:
            ctx.haf_batch(A)
        except gbs.GBSError as e:
            assert e.status == gbs.GBS_EHIP
            print("second call failed as injected")
        else:
            raise SystemExit("no failure injected")
        assert np.allclose(ctx.haf_batch(A).cpu().numpy(), 105, rtol=1e-12)
    """)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    envv = dict(os.environ, GBS_FAULT_INJECT="launch:2", PYTHONPATH=root)
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=envv, capture_output=True, text=True,
                       timeout=180)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "second call failed as injected" in r.stdout


def test_server_fails_only_the_failed_step(env):
    """A served stream with one injected launch failure: the requests of that step fail, every other
    one completes with its alone-run value, and the server keeps serving afterwards."""
    gbs, dev = env
    from paper_1908_10070_amd import serve
    ctx = gbs.Context(0)
    st_in, _ = inputs.config3(count=1)
    st = ctx.state(to_dev(st_in.U, dev), st_in.r)
    rng = np.random.default_rng(8101)
    pats = [inputs.collision_free_patterns(50, int(n), 1, rng)[0] for n in rng.choice([8, 12, 16, 20], size=40)]
    alone = ctx.prob_batch(st, pats).cpu().numpy()
    be = serve.GpuBackend(ctx, st, pool_entries=4096)
    srv = serve.Server(be, pool_entries=4096, step_flops=5e7, max_slice=1024, inflight=1, adaptive=False)
    futs = [srv.submit(p) for p in pats]
    try:
        gbs.debug_fault_inject(3)
        srv.start()
        outcome = []
        for f in futs:
            try:
                outcome.append(f.result(timeout=120))
            except gbs.GBSError as e:
                assert e.status == gbs.GBS_EHIP
                outcome.append(None)
        # serving goes on after the failure
        late = srv.submit(pats[0]).result(timeout=120)
    finally:
        gbs.debug_fault_inject(0)
        srv.stop()
    failed = [i for i, o in enumerate(outcome) if o is None]
    assert 1 <= len(failed) < len(pats)
    assert srv.stats()["failed"] == len(failed) and srv.stats()["steps"] >= 3
    for i, o in enumerate(outcome):
        if o is not None:
            assert o == alone[i], i
    assert late == alone[0]


def test_symmetry_check(env):
    gbs, dev = env
    ctx = gbs.Context(0)
    A_host = inputs.random_symmetric(10, 6, np.random.default_rng(8102))
    A = to_dev(A_host, dev)
    ref = ctx.haf_batch(A).cpu().numpy()
    bad_host = A_host.copy()
    bad_host[3, 2, 7] += 1e-6
    bad = to_dev(bad_host, dev)
    try:
        gbs.debug_check_symmetry(True)
        assert np.array_equal(ctx.haf_batch(A).cpu().numpy(), ref)
        # entries equal up to rounding (a few ulps) pass
        tiny = A_host.copy()
        tiny[1, 0, 5] *= 1 + 4e-16
        ctx.haf_batch(to_dev(tiny, dev))
        with pytest.raises(gbs.GBSError) as ei:
            ctx.haf_batch(bad)
        assert ei.value.status == gbs.GBS_EINVAL and "matrix 3 is not symmetric" in str(ei.value)
        # varlen path: the same matrix found at its position in the call
        ns = np.full(6, 10, dtype=np.int32)
        off = np.arange(6, dtype=np.int64) * 100
        with pytest.raises(gbs.GBSError):
            ctx.haf_batch_varlen(bad.reshape(-1), off, ns)
    finally:
        gbs.debug_check_symmetry(False)
    ctx.haf_batch(bad)  # the check is off again: the call runs
