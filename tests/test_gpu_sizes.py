"""Parity at every supported size, through the C ABI, on general (not structured) inputs.

* n <= 24: random complex-symmetric matrices against the oracle's matching sum (Eq. HafMatch).
* n = 26..46: the same recipe against stored oracle values (tests/golden/general_haf.json, written
  by tests/golden/make_general_golden.py from oracle/ only), each with its cancellation
  kappa = sum_Z |term(Z)| / |Haf| and root-sum-square kappa2 = sqrt(sum_Z |term(Z)|^2) / |Haf|.
* Mixed sizes in one call (haf_batch_varlen and gbs_prob_batch): every engine variant at once.
* The chunk sizes the autotuner can pick: the work-item boundaries move, the results may not.

Tolerance. Up to n = 32 (the sizes of the probability configurations) the bound is 1e-9 relative.
Above, the subset sum cancels strongly (kappa = sum |term| / |Haf| ~ 1e7..1e11), and the bound is
the rounding bound of tests/bounds.py: n^2 u kappa2 with the root-sum-square cancellation kappa2
stored with each value (n^2 u kappa, the worst case, where kappa2 is not stored).
"""
import json
import pathlib

import numpy as np
import pytest
from bounds import U53, bound

import oracle
from paper_1908_10070_amd import inputs

pytestmark = pytest.mark.gpu

GOLD = pathlib.Path(__file__).parent / "golden"
TOL = 1e-9


def load(name):
    p = GOLD / name
    if not p.exists():
        return []
    return json.loads(p.read_text())["records"]


GENERAL = load("general_haf.json")


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


@pytest.fixture(scope="module")
def ctx(torch_dev):
    from paper_1908_10070_amd import gbs
    return gbs.Context(0)


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def relerr(x, ref):
    return float(np.abs(x - ref) / max(abs(ref), 1e-300))


def general_matrix(rec):
    n, count, i = rec["n"], rec["count"], rec["index"]
    return inputs.random_symmetric(n, count, np.random.default_rng(rec["seed"]))[i]


def general_case(rec):
    return f"n{rec['n']}_{rec['index']}"


@pytest.mark.parametrize("rec", GENERAL, ids=[general_case(r) for r in GENERAL])
def test_general_large_n(ctx, torch_dev, rec):
    """n = 26..46 on general complex-symmetric inputs, every kernel instantiation of those k."""
    n = rec["n"]
    A = general_matrix(rec)
    h = ctx.haf_batch(to_dev(A[None], torch_dev)).cpu().numpy()[0]
    ref = complex(*rec["haf"])
    err = relerr(h, ref)
    b = bound(n, rec["kappa"], rec.get("kappa2"), rec["oracle"])
    k2 = rec.get("kappa2", float("nan"))
    print(f"n={n} idx={rec['index']} kappa={rec['kappa']:.2e} kappa2={k2:.2e} err={err:.2e} "
          f"err/(kappa u)={err / (rec['kappa'] * U53):.3f} err/(kappa2 u)={err / (k2 * U53):.2f} bound={b:.2e}")
    assert err <= b, (n, err, b)
    if n <= 32:
        assert err < TOL, (n, err)


def test_general_goldens_cover_every_size():
    """The stored values reach every even n from 26 to 46 (the file is complete)."""
    have = {r["n"] for r in GENERAL}
    missing = [n for n in range(26, 47, 2) if n not in have]
    if missing:
        pytest.skip(f"general_haf.json still lacks n = {missing}")


def test_varlen_every_size_in_one_call(ctx, torch_dev):
    """haf_batch_varlen with a matrix of every n from 0 to 46 (odd ones too) in one call: all 88 engine
    variants run in the same plan, each with its own work counter."""
    import torch
    rng = np.random.default_rng(4600)
    mats, refs, tols = [], [], []
    by_n = {}
    for r in GENERAL:
        by_n.setdefault(r["n"], r)
    for n in range(0, 47):
        if n >= 26 and n % 2 == 0:
            rec = by_n.get(n)
            if rec is None:
                continue
            A = general_matrix(rec)
            refs.append(complex(*rec["haf"]))
            tols.append(max(TOL, bound(n, rec["kappa"], rec.get("kappa2"), rec["oracle"])))
        else:
            A = inputs.random_symmetric(n, 1, rng)[0] if n else np.zeros((0, 0), np.complex128)
            refs.append(oracle.haf_enum(A) if n <= 25 else 0j)
            tols.append(TOL)
        mats.append(A)
    ns = np.array([a.shape[0] for a in mats], dtype=np.int32)
    off = np.zeros(len(mats), dtype=np.int64)
    off[1:] = np.cumsum([a.size for a in mats[:-1]])
    flat = np.concatenate([a.reshape(-1) for a in mats] + [np.zeros(1, np.complex128)])
    A_dev = torch.from_numpy(flat).to(torch_dev)
    h = ctx.haf_batch_varlen(A_dev, off, ns).cpu().numpy()
    for i, n in enumerate(ns):
        if n % 2:
            assert h[i] == 0, n
        elif n == 0:
            assert h[i] == 1
        else:
            err = relerr(h[i], refs[i])
            assert err <= tols[i], (int(n), err, tols[i])
    # every result equals the same matrix evaluated alone
    for i in (2, 10, 24, len(mats) - 1):
        alone = ctx.haf_batch_varlen(A_dev, off[i:i + 1], ns[i:i + 1]).cpu().numpy()[0]
        assert alone == h[i], int(ns[i])


def test_prob_batch_mixed_sizes(ctx, torch_dev):
    """gbs_prob_batch with patterns of n = 2..24 (random, some with repeated modes) and the config-5
    patterns that have stored values, on the config-5 state, in one call."""
    st_in, pats5 = inputs.config5()
    st = ctx.state(to_dev(st_in.U, torch_dev), st_in.r)
    B = oracle.state_B(st_in.U, st_in.r)
    pref = float(np.prod(1.0 / np.cosh(st_in.r)))
    rng = np.random.default_rng(4601)
    pats, refs, tols = [], [], []
    for n in range(2, 25, 2):
        p = sorted(rng.choice(60, n, replace=False).tolist())
        if n % 4 == 0:
            p[1] = p[0]  # one collision
        pats.append(p)
        refs.append(oracle.prob_ref(st_in.U, st_in.r, p))
        tols.append(TOL)
    for rec in load("config5_haf.json"):
        if "kappa" not in rec:
            continue
        p = [int(v) for v in pats5[rec["index"]]]
        assert p == rec["modes"]
        ld = "haf_pt_ld" in rec
        h = complex(*(rec["haf_pt_ld"] if ld else rec["haf_pt"]))
        pats.append(p)
        refs.append(abs(h) ** 2 * pref)
        # p = |Haf|^2 pref: twice the hafnian's relative error
        tols.append(2 * bound(len(p), rec["kappa"], rec.get("kappa2"), "long double" if ld else "double"))
    prob = ctx.prob_batch(st, pats).cpu().numpy()
    for i, p in enumerate(pats):
        err = relerr(prob[i], refs[i])
        assert err <= tols[i], (len(p), err, tols[i])
    del B


@pytest.mark.parametrize("n,shape", [(24, 1), (24, 2), (24, 3), (30, 3), (38, 1), (38, 2), (22, 4), (24, 8), (24, 12),
                                     (26, 12), (30, 4), (34, 8), (38, 4), (38, 12), (46, 12), (26, 16), (28, 20),
                                     (32, 16), (36, 20), (40, 16), (42, 20), (44, 20), (46, 20)])
def test_engine_shapes(ctx, torch_dev, n, shape):
    """The engine shapes the autotuner can pick (|Z| = 9, 10 and / or 11, 12 on the 16x16-tile engine or
    the symmetric quad-tile engine; |Z| = 13, 14 on the 7x7 symmetric quad-tile engine) give the oracle's values (n <= 24 against the matching sum; larger n
    against the stored ones) and agree with the built-in shape up to the order of the partial sums."""
    from paper_1908_10070_amd import gbs
    if n <= 24:
        A = inputs.random_symmetric(n, 8, np.random.default_rng(5100 + n))
        refs = [oracle.haf_enum(a) for a in A]
        tols = [TOL] * len(A)
    else:
        recs = [r for r in GENERAL if r["n"] == n]
        if not recs:
            pytest.skip(f"no stored value for n = {n}")
        A = np.stack([general_matrix(r) for r in recs])
        refs = [complex(*r["haf"]) for r in recs]
        tols = [max(TOL, bound(n, r["kappa"], r.get("kappa2"), r["oracle"])) for r in recs]
    A_dev = to_dev(A, torch_dev)
    c = gbs.Context(0)
    c.set_shape(n, shape)
    assert c.get_shape(n) == shape
    h = c.haf_batch(A_dev).cpu().numpy()
    base = ctx.haf_batch(A_dev).cpu().numpy()
    for i in range(len(A)):
        assert relerr(h[i], refs[i]) <= tols[i], (n, shape, i)
        assert relerr(h[i], base[i]) <= max(1e-11, 2 * tols[i]), (n, shape, i)
    # the no-allocation entry point follows the same shape
    import torch
    out = torch.empty(len(A), dtype=torch.complex128, device=torch_dev)
    assert np.array_equal(c.haf_batch_noalloc(A_dev, out).cpu().numpy(), h)
    c.set_shape(n, -1)
    assert c.get_shape(n) == ctx.get_shape(n)  # back to the built-in table
    with pytest.raises(gbs.GBSError):
        c.set_shape(n, 32)


@pytest.mark.parametrize("chunks", [(512, 256), (2048, 16), (128, 8), (4096, 128)])
def test_tuned_chunk_sizes(torch_dev, chunks):
    """The headline workload (config 2, n = 24) at chunk pairs the autotuner can pick: oracle parity
    on a sample, and the same results as at the built-in chunks up to the order of the partial sums."""
    from paper_1908_10070_amd import gbs
    A = inputs.config2()[:512]
    A_dev = to_dev(A, torch_dev)
    c = gbs.Context(0)
    c.set_tuning(24, *chunks)
    assert c.get_tuning(24) == tuple(chunks)
    h = c.haf_batch(A_dev).cpu().numpy()
    idx = np.concatenate([[0, 1, 511], np.random.default_rng(9).choice(512, 9, replace=False)])
    for i in idx:
        assert relerr(h[i], oracle.haf_enum(A[i])) < TOL, (chunks, int(i))
    base = gbs.Context(0).haf_batch(A_dev).cpu().numpy()
    assert np.max(np.abs(h - base) / np.abs(base)) < 1e-11
    # replaying the captured graph gives the same bits
    h2 = c.haf_batch(A_dev).cpu().numpy()
    assert np.array_equal(h, h2)
