"""The entry point that allocates nothing (haf_batch_noalloc), through the C ABI, against haf_batch.

Its plan is built on the device from the same per-pattern work items haf_batch stages from the host,
and it runs the same kernels and summation order, so at the same chunk sizes its results must equal
haf_batch's bit for bit; they are also checked against the oracle (1e-9). Two calls in a row, the
second with a smaller input, share the one static scratch array."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1908_10070_amd import gbs, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def call_noalloc(ctx, A, out):
    """haf_batch_noalloc through the C ABI (ctypes, no binding helper)."""
    import torch
    b, n = A.shape[0], A.shape[1]
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return gbs.lib().haf_batch_noalloc(ctx.handle, ctypes.c_void_p(A.data_ptr()), n, b, n * n,
                                       ctypes.c_void_p(out.data_ptr()), s)


def test_noalloc_matches_haf_batch_twice(torch_dev):
    import torch
    ctx = gbs.Context(0)
    rng = np.random.default_rng(77)
    cases = [(20, 300), (24, 96), (16, 7)]  # second and third calls smaller than the first
    for n, batch in cases:
        A = inputs.random_symmetric(n, batch, rng)
        A_dev = torch.from_numpy(A).to(torch_dev)
        out = torch.full((batch,), complex(7.0, -7.0), dtype=torch.complex128, device=torch_dev)
        assert call_noalloc(ctx, A_dev, out) == gbs.GBS_OK, gbs.lib().gbs_last_error(ctx.handle)
        ref = ctx.haf_batch(A_dev)
        torch.cuda.synchronize()
        got, ref = out.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(got, ref), (n, batch, np.max(np.abs(got - ref)))
        for i in (0, batch // 2, batch - 1):
            h = oracle.haf_enum(A[i])
            assert abs(got[i] - h) <= 1e-9 * abs(h), (n, i)


def test_noalloc_edge_sizes_and_limit(torch_dev):
    import torch
    ctx = gbs.Context(0)
    # n = 0 (every result 1) and odd n (0), through the device-built plan with no work items
    for n, want in ((0, 1), (5, 0)):
        A_dev = torch.zeros((3, n, n), dtype=torch.complex128, device=torch_dev)
        out = torch.full((3,), complex(7.0, -7.0), dtype=torch.complex128, device=torch_dev)
        assert call_noalloc(ctx, A_dev, out) == gbs.GBS_OK
        torch.cuda.synchronize()
        assert np.all(out.cpu().numpy() == want), n
    # a plan beyond the scratch (n = 46 cut into items of 8 subsets: about 1M items and partials,
    # ~60 MB against 32 MiB): rejected, nothing enqueued, the output untouched
    ctx.set_tuning(46, 8, 8)
    A_dev = torch.zeros((1, 46, 46), dtype=torch.complex128, device=torch_dev)
    out = torch.full((1,), complex(7.0, -7.0), dtype=torch.complex128, device=torch_dev)
    assert call_noalloc(ctx, A_dev, out) == gbs.GBS_ENOMEM
    assert b"no-allocation scratch" in gbs.lib().gbs_last_error(ctx.handle)
    torch.cuda.synchronize()
    assert out.cpu().numpy()[0] == complex(7.0, -7.0)
