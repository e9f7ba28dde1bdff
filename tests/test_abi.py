"""CPU checks of the C ABI: the library loads, exports what include/gbs.h declares, and its
host-only entry points behave (no GPU compute is called here)."""
import ctypes
import pathlib
import re

import pytest

from paper_1908_10070_amd import gbs

ROOT = pathlib.Path(__file__).resolve().parents[1]


def header_functions():
    text = (ROOT / "include" / "gbs.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


@pytest.fixture(scope="module")
def lib():
    if not gbs.LIB_PATH.exists():
        from paper_1908_10070_amd.csrc import build
        build.build(force=False)
    return gbs.lib()


def test_header_functions_parsed():
    fns = header_functions()
    assert "gbs_prob_batch" in fns and "haf_batch" in fns and len(fns) >= 15


def test_every_declared_symbol_is_exported(lib):
    for name in header_functions():
        assert hasattr(lib, name), name
    assert sorted(gbs.EXPORTS) == header_functions()


def test_status_strings(lib):
    for s in range(6):
        assert lib.gbs_status_str(s)
    assert lib.gbs_status_str(99) == b"unknown status"


def test_subset_count_and_flops(lib):
    assert gbs.subset_count(0) == 0
    assert gbs.subset_count(3) == 0
    assert gbs.subset_count(24) == 4095
    assert gbs.subset_count(44) == 2 ** 22 - 1
    assert gbs.subset_count(gbs.GBS_N_MAX + 2) == 0
    # the flop model of the power-trace method as formulated (every subset, all k traces, chain for k:
    # products + inner products + coefficient recursion). n = 8 (k = 4: 1 product, 2 inner products):
    # |Z|=1: 4 x (8*8 + 2*8*4 + 80) = 832;  |Z|=2: 6 x (8*64 + 2*8*16 + 80) = 5088
    # |Z|=3: 4 x (8*216 + 2*8*36 + 80) = 9536;  |Z|=4: 8*512 + 2*8*64 + 80 = 5200
    assert gbs.haf_flops(8) == 832 + 5088 + 9536 + 5200
    assert abs(gbs.haf_flops(24) - 3.215e8) / 3.215e8 < 2e-3
    assert gbs.haf_flops(7) == 0.0


def test_null_context_rejected(lib):
    vp = ctypes.c_void_p
    assert lib.haf_batch(None, None, 4, 1, 16, None, None) == gbs.GBS_EINVAL
    assert lib.gbs_prob_batch(None, None, None, None, 1, None, None, None) == gbs.GBS_EINVAL
    assert lib.gbs_ctx_destroy(None) == gbs.GBS_EINVAL
    assert lib.gbs_state_destroy(None) == gbs.GBS_EINVAL
    assert lib.gbs_ctx_set_exec(None, 1, 1) == gbs.GBS_EINVAL
    assert lib.gbs_ctx_set_streams(None, 2) == gbs.GBS_EINVAL
    assert lib.gbs_ctx_get_streams(None, None) == gbs.GBS_EINVAL
    out = vp()
    assert lib.gbs_ctx_create(0, None, 0, None) == gbs.GBS_EINVAL
    assert lib.gbs_ctx_create(0, None, 123, ctypes.byref(out)) == gbs.GBS_EINVAL


def test_pack_patterns():
    import numpy as np
    modes, off = gbs.pack_patterns([[1, 2], [], [3, 4, 5, 6]])
    assert modes.tolist() == [1, 2, 3, 4, 5, 6] and off.tolist() == [0, 2, 2, 6]
    modes, off = gbs.pack_patterns(np.array([[0, 1], [2, 3]]))
    assert off.tolist() == [0, 2, 4]


def test_photon_number_pmf_matches_oracle():
    """Step 1's table is host code in the library: P_n against the oracle's closed form."""
    import oracle
    from paper_1908_10070_amd import gbs
    for m, r in [(16, 0.5), (36, 0.3423), (5, 0.8814)]:
        p = gbs.photon_number_pmf(m, r, 60)
        for n in range(61):
            assert abs(p[n] - oracle.photon_number_prob(m, n, r)) <= 1e-12 * max(p[n], 1e-300) + 1e-300
    assert abs(gbs.photon_number_pmf(36, 0.3423, 400).sum() - 1.0) < 1e-12


def test_sweep_count():
    """Number of output patterns: C(m + n - 1, n) with collisions, C(m, n) without; -1 past the limits."""
    import math
    for m, n in [(16, 8), (5, 4), (1, 3), (7, 0), (30, 10)]:
        assert gbs.sweep_count(m, n, True) == math.comb(m + n - 1, n)
        assert gbs.sweep_count(m, n, False) == math.comb(m, n)
    assert gbs.sweep_count(50, 20, True) == -1  # beyond 2^31 - 1 patterns
    assert gbs.sweep_count(4, 33, True) == -1   # n beyond the sweep's limit
    assert gbs.sweep_count(0, 2, True) == -1


def test_precision_null_context():
    """gbs_ctx_set_precision / gbs_ctx_get_precision reject a null context without touching a device."""
    from paper_1908_10070_amd import gbs
    L = gbs.lib()
    assert L.gbs_ctx_set_precision(None, gbs.GBS_PREC_DD) == gbs.GBS_EINVAL
    assert L.gbs_ctx_get_precision(None) == gbs.GBS_PREC_FP64
