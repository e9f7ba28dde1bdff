"""Autotuner: cache round trip (CPU) and a quick measured tuning (GPU)."""
import json

import numpy as np
import pytest

from paper_1908_10070_amd import autotune


class FakeCtx:
    def __init__(self):
        self.t = {}
        self.sh = {}

    def set_tuning(self, n, cs, cl):
        self.t[n] = (cs, cl)

    def set_shape(self, n, shape):
        self.sh[n] = shape


def test_cache_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    autotune.save_cache({("gfx950", 24): (512, 16), ("gfx942", 24): (1024, 32)}, path)
    autotune.save_cache({("gfx950", 20): (256, 8), ("gfx950", 30): (512, 32, 3)}, path)
    data = json.loads(path.read_text())
    assert data["gfx950:24"] == {"chunk_small": 512, "chunk_large": 16}
    assert data["gfx950:20"]["chunk_small"] == 256
    assert data["gfx950:30"] == {"chunk_small": 512, "chunk_large": 32, "shape": 3}
    ctx = FakeCtx()
    monkeypatch.setattr(autotune, "_arch", lambda c: "gfx950")
    assert autotune.load_cache(ctx, path) == 3
    assert ctx.t == {24: (512, 16), 20: (256, 8), 30: (512, 32)}
    assert ctx.sh == {30: 3}


def test_shapes_for():
    """Only engine choices that apply at n are searched: |Z| = 9, 10 from k = 9 (symmetric quad-tile
    from k = 11), |Z| = 11, 12 from k = 11, |Z| = 13, 14 from k = 13."""
    assert autotune.shape_bands(16) == []
    assert autotune.shapes_for(16) == (0,)
    assert autotune.shapes_for(18) == (0, 1)
    assert autotune.shape_bands(22) == [[0, 1, 8], [0, 2, 4]]
    assert sorted(autotune.shapes_for(22)) == [0, 1, 2, 3, 4, 5, 8, 10, 12]
    assert autotune.shape_bands(24) == [[0, 1, 8], [0, 2, 4]]
    assert autotune.shape_bands(26) == [[0, 1, 8], [0, 2, 4], [0, 16]]
    assert autotune.shape_bands(46) == [[0, 1, 8], [0, 2, 4], [0, 16]]
    assert len(autotune.shapes_for(46)) == 18 and 20 in autotune.shapes_for(46)


def test_ties_go_to_the_smaller_chunk():
    assert autotune.smallest_within({128: 10.05, 256: 10.0, 512: 9.98}) == 128
    assert autotune.smallest_within({128: 10.5, 256: 10.0, 512: 9.98}) == 256
    assert autotune.smallest_within({64: 3.0}) == 64
    assert autotune.smallest_within({8: 2.0, 16: 1.0}, tol=0.0) == 16


def test_engine_changes_only_when_clearly_faster():
    assert autotune.faster_than(4, {4: 10.0, 20: 9.95, 0: 10.2}) == 4
    assert autotune.faster_than(4, {4: 10.0, 20: 9.8, 0: 10.2}) == 20
    assert autotune.faster_than(0, {0: 10.0, 2: 10.5}) == 0


def test_load_cache_missing_or_corrupt(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "_arch", lambda c: "gfx950")
    assert autotune.load_cache(FakeCtx(), tmp_path / "none.json") == 0
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    assert autotune.load_cache(FakeCtx(), bad) == 0


@pytest.mark.gpu
def test_tune_on_device(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_10070_amd import gbs, inputs
    import oracle
    ctx = gbs.Context(0)
    A_host = inputs.random_symmetric(18, 256, np.random.default_rng(9))
    A = torch.from_numpy(A_host).cuda()
    log = []
    cs, cl = autotune.tune(ctx, 18, A, reps=1, small=(64, 256), large=(8, 32), cache=tmp_path / "t.json", log=log)
    assert (cs, cl) == ctx.get_tuning(18) and len(log) == 6  # 2 + 2 chunk trials, shapes 1 and 0
    assert ctx.get_shape(18) in (0, 1)
    assert json.loads((tmp_path / "t.json").read_text())
    h = ctx.haf_batch(A).cpu().numpy()
    for i in (0, 100, 255):
        ref = oracle.haf_enum(A_host[i])
        assert abs(h[i] - ref) <= 1e-9 * abs(ref)
