"""Parity of the HIP path with the CPU oracle, called through the C ABI (gfx950 only).

Tolerance: relative error 1e-9 on hafnians and probabilities (complex128 throughout).
"""
import json
import math
import pathlib

import bounds
import numpy as np
import pytest

import oracle
from paper_1908_10070_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-9


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
    x = np.asarray(x)
    ref = np.asarray(ref)
    return np.abs(x - ref) / np.maximum(np.abs(ref), 1e-300)


def dfact(n):
    return math.prod(range(n - 1, 0, -2)) if n > 0 else 1


def test_state_B_and_prefactor(ctx, torch_dev):
    st_in, _ = inputs.config1()
    st = ctx.state(to_dev(st_in.U, torch_dev), st_in.r)
    B = st.B().cpu().numpy()
    Bref = oracle.state_B(st_in.U, st_in.r)
    assert np.max(np.abs(B - Bref)) < 1e-14
    assert abs(st.prefactor - 0.1463386077562255) < 1e-16


@pytest.mark.parametrize("n", list(range(0, 25)) + [26, 28])
def test_haf_sizes_vs_oracle(ctx, torch_dev, n):
    """Every size up to 24 (odd ones give 0), a few beyond: several tiles and ragged tails."""
    rng = np.random.default_rng(100 + n)
    A = inputs.random_symmetric(n, 3, rng)
    h = ctx.haf_batch(to_dev(A, torch_dev)).cpu().numpy()
    for i in range(3):
        ref = oracle.haf_enum(A[i]) if n <= 24 else oracle.haf_pt_ld(A[i])
        if n % 2:
            assert h[i] == 0
        elif n == 0:
            assert h[i] == 1
        else:
            assert relerr(h[i], ref) < TOL, (n, i, h[i], ref)


def test_config1_full(ctx, torch_dev):
    """m = 16, r = 0.5: all 12,870 collision-free 8-photon patterns plus the vacuum."""
    st_in, pats = inputs.config1()
    st = ctx.state(to_dev(st_in.U, torch_dev), st_in.r)
    allp = [[]] + [list(p) for p in pats]
    prob, haf = ctx.prob_batch(st, allp, want_haf=True)
    prob, haf = prob.cpu().numpy(), haf.cpu().numpy()
    href = oracle.haf_ref_patterns(st_in.U, st_in.r, pats)
    pref = oracle.prob_ref_patterns(st_in.U, st_in.r, pats)
    assert abs(prob[0] - 0.1463386077562255) < 1e-16
    assert haf[0] == 1
    assert np.max(relerr(haf[1:], href)) < TOL
    assert np.max(relerr(prob[1:], pref)) < TOL


def test_config2_sampled(ctx, torch_dev):
    """4096 random complex-symmetric 24 x 24 matrices; oracle on a seeded sample."""
    A = inputs.config2()
    h = ctx.haf_batch(to_dev(A, torch_dev)).cpu().numpy()
    idx = np.random.default_rng(5).choice(len(A), 24, replace=False)
    idx = np.concatenate([[0, len(A) - 1], idx])
    ref = np.array([oracle.haf_enum(A[i]) for i in idx])
    err = relerr(h[idx], ref)
    assert np.max(err) < TOL, err


def test_collisions(ctx, torch_dev):
    rng = np.random.default_rng(11)
    m = 10
    U = inputs.haar_unitary(m, rng)
    r = rng.uniform(0.2, 0.9, size=m)
    st = ctx.state(to_dev(U, torch_dev), r)
    pats = [[0, 0], [1, 1, 1, 1], [2, 3, 3, 4], [5, 5, 6, 6, 7, 7], [9, 0, 9, 0, 1, 2, 3, 3], [4, 4, 4], [8]]
    prob, haf = ctx.prob_batch(st, pats, want_haf=True)
    prob, haf = prob.cpu().numpy(), haf.cpu().numpy()
    for i, p in enumerate(pats):
        ref = oracle.prob_ref(U, r, p)
        if len(p) % 2:
            assert prob[i] == 0 and haf[i] == 0
        else:
            assert relerr(prob[i], ref) < TOL, p
            assert relerr(haf[i], oracle.haf_enum(oracle.pattern_matrix(oracle.state_B(U, r), p))) < TOL


def test_all_ones_closed_form(ctx, torch_dev):
    import torch
    for n in (2, 8, 16, 18, 24, 32):
        A = torch.ones((1, n, n), dtype=torch.complex128, device=torch_dev)
        h = ctx.haf_batch(A).cpu().numpy()[0]
        assert relerr(h, dfact(n)) < TOL, n


def test_bipartite_is_permanent(ctx, torch_dev):
    """Haf([[0, W], [W^t, 0]]) = Per(W) (Ryser's formula, vectorised, as the reference)."""
    for k in (5, 9, 12, 14, 16):
        rng = np.random.default_rng(200 + k)
        W = (rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))) / np.sqrt(2)
        A = np.block([[np.zeros((k, k)), W], [W.T, np.zeros((k, k))]])
        h = ctx.haf_batch(to_dev(A[None], torch_dev)).cpu().numpy()[0]
        masks = np.arange(1, 1 << k)
        sel = ((masks[:, None] >> np.arange(k)[None, :]) & 1).astype(np.float64)
        rows = sel @ W.T  # (2^k-1, k): row sums over selected columns
        signs = (-1.0) ** sel.sum(axis=1)
        per = (-1) ** k * np.sum(signs * np.prod(rows, axis=1))
        assert relerr(h, per) < TOL, k


def test_batch_composition_is_bitwise_invariant(ctx, torch_dev):
    """A pattern's result does not depend on what else is in the batch, nor on the launch mode."""
    from paper_1908_10070_amd import gbs
    rng = np.random.default_rng(21)
    A = inputs.random_symmetric(20, 6, rng)
    full = ctx.haf_batch(to_dev(A, torch_dev)).cpu().numpy()
    alone = np.array([ctx.haf_batch(to_dev(A[i:i + 1], torch_dev)).cpu().numpy()[0] for i in range(6)])
    assert np.array_equal(full, alone)
    for use_graph, persistent in [(False, True), (False, False), (True, False)]:
        c2 = gbs.Context(0, use_graph=use_graph, persistent=persistent)
        assert np.array_equal(c2.haf_batch(to_dev(A, torch_dev)).cpu().numpy(), full)


def test_multi_stream_launches_are_bitwise_equal(ctx, torch_dev):
    """Spreading a mixed batch's kernels over several streams changes only their overlap."""
    from paper_1908_10070_amd import gbs
    rng = np.random.default_rng(24)
    m = 40
    U = inputs.haar_unitary(m, rng)
    r = np.full(m, 0.88)
    st = ctx.state(to_dev(U, torch_dev), r)
    pats = [sorted(rng.choice(m, int(n), replace=False).tolist()) for n in rng.choice(range(4, 31, 2), 60)]
    ref = ctx.prob_batch(st, pats).cpu().numpy()
    assert gbs.Context(0).streams == 2  # a new context's default
    for ns, graph, persistent in [(4, False, True), (8, False, False), (3, False, True), (4, True, True),
                                  (8, True, False)]:
        c2 = gbs.Context(0, use_graph=graph, persistent=persistent)
        c2.set_streams(ns)
        assert c2.streams == ns
        for _ in range(3):  # a graph is captured on the first call and replayed after
            assert np.array_equal(c2.prob_batch(st, pats).cpu().numpy(), ref), (ns, graph)
    with pytest.raises(gbs.GBSError):
        c2.set_streams(9)
    # a one-size batch on a context left at its default takes the built-in count for its n (one
    # stream at n = 20, two at n = 24): the same bits as either explicit count
    for n in (20, 24):
        pn = [sorted(rng.choice(m, n, replace=False).tolist()) for _ in range(24)]
        ref_n = gbs.Context(0).prob_batch(st, pn).cpu().numpy()
        for ns in (1, 2):
            c3 = gbs.Context(0)
            c3.set_streams(ns)
            assert np.array_equal(c3.prob_batch(st, pn).cpu().numpy(), ref_n), (n, ns)


def test_graph_replays(ctx, torch_dev):
    import torch
    rng = np.random.default_rng(22)
    A = to_dev(inputs.random_symmetric(16, 40, rng), torch_dev)
    out = torch.empty(40, dtype=torch.complex128, device=torch_dev)
    ref = ctx.haf_batch(A, out=out).clone()
    for _ in range(4):
        out.zero_()
        torch.cuda.synchronize()
        ctx.haf_batch(A, out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


def test_reused_plan_storage_across_call_shapes(torch_dev):
    """A context keeps its plan storage between calls: a large one-size batch, then a small mixed one,
    sliced subset ranges, a one-size batch of another n and the large batch again on one context give
    the bits that each call gives on a fresh context."""
    from paper_1908_10070_amd import gbs
    rng = np.random.default_rng(31)
    m = 40
    U = inputs.haar_unitary(m, rng)
    big = [sorted(rng.choice(m, 20, replace=False).tolist()) for _ in range(3000)]
    mixed = [sorted(rng.choice(m, int(n), replace=False).tolist()) for n in rng.choice(range(0, 29, 2), 50)]
    other = [sorted(rng.choice(m, 24, replace=False).tolist()) for _ in range(40)]
    c = gbs.Context(0)
    st = c.state(to_dev(U, torch_dev), np.full(m, 0.88))

    def fresh(pats):
        return gbs.Context(0).prob_batch(st, pats).cpu().numpy()

    expect = {name: fresh(p) for name, p in (("big", big), ("mixed", mixed), ("other", other))}
    assert np.array_equal(c.prob_batch(st, big).cpu().numpy(), expect["big"])
    assert np.array_equal(c.prob_batch(st, mixed).cpu().numpy(), expect["mixed"])
    # each n = 24 pattern's subset range in two uneven slices, combined by finalize (the same value to
    # rounding: the slices' partials are summed in another order than one item list's)
    total = gbs.subset_count(24)
    sl_pats = [p for p in other for _ in range(2)]
    lo = [v for _ in other for v in (0, total // 3)]
    hi = [v for _ in other for v in (total // 3, total)]
    parts = c.prob_slices(st, sl_pats, lo, hi)
    offs = list(range(0, 2 * len(other) + 1, 2))
    p_sl, _ = c.finalize(st, parts, offs[:-1], offs[1:], other)
    assert np.max(relerr(p_sl.cpu().numpy(), expect["other"])) < TOL
    assert np.array_equal(c.prob_batch(st, other).cpu().numpy(), expect["other"])
    assert np.array_equal(c.prob_batch(st, big).cpu().numpy(), expect["big"])


def test_slices_and_finalize(ctx, torch_dev):
    from paper_1908_10070_amd import gbs
    rng = np.random.default_rng(23)
    m = 30
    U = inputs.haar_unitary(m, rng)
    r = np.full(m, 0.88)
    st = ctx.state(to_dev(U, torch_dev), r)
    pats = [sorted(rng.choice(m, n, replace=False).tolist()) for n in (18, 22, 12)]
    prob = ctx.prob_batch(st, pats).cpu().numpy()
    # cut each pattern's subset range into uneven slices
    sl_pats, lo, hi, part_off = [], [], [], [0]
    for p in pats:
        cnt = gbs.subset_count(len(p))
        cuts = sorted(set([0, cnt] + rng.integers(0, cnt, 4).tolist()))
        for a, b in zip(cuts[:-1], cuts[1:]):
            sl_pats.append(p)
            lo.append(a)
            hi.append(b)
        part_off.append(part_off[-1] + len(cuts) - 1)
    parts = ctx.prob_slices(st, sl_pats, lo, hi)
    p2, h2 = ctx.finalize(st, parts, part_off[:-1], part_off[1:], pats)
    assert np.max(relerr(p2.cpu().numpy(), prob)) < TOL


def test_invalid_inputs_raise(ctx, torch_dev):
    from paper_1908_10070_amd import gbs
    st_in, _ = inputs.config1()
    st = ctx.state(to_dev(st_in.U, torch_dev), st_in.r)
    with pytest.raises(gbs.GBSError) as e:
        ctx.prob_batch(st, [[0, 16]])
    assert e.value.status == gbs.GBS_ERANGE
    with pytest.raises(gbs.GBSError) as e:
        ctx.prob_batch(st, [list(range(16)) * 4])
    assert e.value.status == gbs.GBS_ERANGE
    with pytest.raises(ValueError):
        ctx.prob_batch(st, (np.array([0, 1], np.int32), np.array([0, 3], np.int64)))
    with pytest.raises(gbs.GBSError) as e:
        ctx.prob_batch(st, (np.array([0, 1, 2], np.int32), np.array([0, 2, 1], np.int64)))
    assert e.value.status == gbs.GBS_EINVAL


@pytest.mark.parametrize("k", [17, 18, 19, 20, 21, 22, 23])
def test_bipartite_permanent_large(ctx, torch_dev, k):
    """n = 34..46: Haf of the bipartite block matrix [[0, W], [W^t, 0]] against the permanent of W by
    Ryser's formula (an independent closed form) and against the oracle's power trace stored by
    tests/golden/make_general_golden.py --bipartite. Tolerances: the rounding bound of tests/bounds.py
    from the stored kappa, kappa2 of the subset sum; against Ryser's double sum, plus its own bound
    2 k u kappa_R (k - 1 additions per row sum and k - 1 products per term, each within u), with
    kappa_R of Ryser's alternating sum (worst case sum |term|, root-sum-square counterpart as in
    tests/bounds.py; the tighter)."""
    recs = {}
    path = pathlib.Path(__file__).parent / "golden" / "bipartite_haf.json"
    if path.exists():
        recs = {r["k"]: r for r in json.loads(path.read_text())["records"]}
    if k not in recs:
        pytest.skip(f"no stored oracle value for k = {k}")
    g = recs[k]
    n = 2 * k
    W, A = inputs.bipartite(k, np.random.default_rng(300 + k))
    h = ctx.haf_batch(to_dev(A[None], torch_dev)).cpu().numpy()[0]
    per = 0j
    s1 = 0.0
    s2 = 0.0
    step = 1 << 16
    cols = np.arange(k)
    for s0 in range(1, 1 << k, step):
        masks = np.arange(s0, min(1 << k, s0 + step))
        sel = ((masks[:, None] >> cols[None, :]) & 1).astype(np.float64)
        terms = (-1.0) ** sel.sum(axis=1) * np.prod(sel @ W.T, axis=1)
        per += np.sum(terms)
        s1 += float(np.sum(np.abs(terms)))
        s2 += float(np.sum(np.abs(terms) ** 2))
    per *= (-1) ** k
    ryser = 2 * k * bounds.U53 * min(s1, np.sqrt(s2)) / abs(per)
    b = bounds.bound(n, g["kappa"], g["kappa2"], g["oracle"])
    ref = complex(*g["haf"])
    print(f"k={k} n={n} vs Ryser {relerr(h, per):.3e} (bound {b + ryser:.2e}), vs oracle {relerr(h, ref):.3e} "
          f"(bound {b:.2e})")
    assert relerr(h, ref) <= b
    assert relerr(h, per) <= bounds.bound(n, g["kappa"], g["kappa2"]) + ryser


def test_config5_large_hafnians_vs_oracle_goldens(ctx, torch_dev):
    """Config 5 (m = 60, r = 0.88, n = 36/40/44 B_S submatrices) in one batched call, against the
    oracle's power trace stored by tests/golden/make_config5_golden.py (long double where present,
    else double) with each matrix's cancellation kappa = sum_Z |term(Z)| / |Haf| (and kappa2, its
    root-sum-square counterpart). Bound: the rounding bound of tests/bounds.py."""
    gold = json.loads((pathlib.Path(__file__).parent / "golden" / "config5_haf.json").read_text())["records"]
    gold = [g for g in gold if "kappa" in g]
    if not gold:
        pytest.skip("no config-5 record with kappa yet")
    st_in, pats = inputs.config5()
    st = ctx.state(to_dev(st_in.U, torch_dev), st_in.r)
    sel = [pats[g["index"]] for g in gold]
    for g, p in zip(gold, sel):
        assert [int(v) for v in p] == g["modes"]
    prob, haf = ctx.prob_batch(st, sel, want_haf=True)
    haf = haf.cpu().numpy()
    for g, h in zip(gold, haf):
        ld = "haf_pt_ld" in g
        ref = complex(*(g["haf_pt_ld"] if ld else g["haf_pt"]))
        err = relerr(h, ref)
        b = bounds.bound(g["n"], g["kappa"], g.get("kappa2"), "long double" if ld else "double")
        print(f"config5 index {g['index']} n={g['n']} kappa={g['kappa']:.2e} kappa2={g.get('kappa2', float('nan')):.2e} "
              f"rel err {err:.2e} vs {'long double' if ld else 'double'} oracle, bound {b:.2e}")
        assert err <= b, (g["index"], err, b)


def test_config5_slices_vs_oracle_goldens(ctx, torch_dev):
    """Config-5 patterns of n = 36, 40 and 44 cut into uneven subset slices (slice edges inside every
    engine band: the 6x6 and 7x7 symmetric quad-tile kernels, the 16x16-tile kernels, the quad grids),
    evaluated by gbs_prob_slices and combined by gbs_finalize, against the stored oracle values with
    the same rounding bound as the batched call."""
    from paper_1908_10070_amd import gbs
    gold = json.loads((pathlib.Path(__file__).parent / "golden" / "config5_haf.json").read_text())["records"]
    picked = {}
    for g in gold:
        if "kappa" in g and g["n"] not in picked:
            picked[g["n"]] = g
    gold = [picked[n] for n in sorted(picked)]
    if not gold:
        pytest.skip("no config-5 record with kappa yet")
    st_in, pats = inputs.config5()
    st = ctx.state(to_dev(st_in.U, torch_dev), st_in.r)
    rng = np.random.default_rng(55)
    sl_pats, lo, hi, part_off = [], [], [], [0]
    for g in gold:
        p = pats[g["index"]]
        cnt = gbs.subset_count(len(p))
        cuts = sorted(set([0, cnt] + rng.integers(1, cnt, 7).tolist()))
        for a, b in zip(cuts[:-1], cuts[1:]):
            sl_pats.append(p)
            lo.append(a)
            hi.append(b)
        part_off.append(part_off[-1] + len(cuts) - 1)
    parts = ctx.prob_slices(st, sl_pats, lo, hi)
    _, haf = ctx.finalize(st, parts, part_off[:-1], part_off[1:], [pats[g["index"]] for g in gold])
    haf = haf.cpu().numpy()
    for g, h in zip(gold, haf):
        ld = "haf_pt_ld" in g
        ref = complex(*(g["haf_pt_ld"] if ld else g["haf_pt"]))
        b = bounds.bound(g["n"], g["kappa"], g.get("kappa2"), "long double" if ld else "double")
        assert relerr(h, ref) <= b, (g["index"], g["n"], relerr(h, ref), b)


def test_config3_full_size_sampled(ctx, torch_dev):
    """Config 3 as the benchmark runs it (100,000 twenty-photon patterns, m = 50, one batched call):
    40 outputs spread over the batch against the oracle, and properties of all of them."""
    st_in, pats = inputs.config3()
    st = ctx.state(to_dev(st_in.U, torch_dev), st_in.r)
    prob = ctx.prob_batch(st, pats).cpu().numpy()
    assert prob.shape == (len(pats),) and np.all(np.isfinite(prob)) and np.all(prob > 0)
    # distinct collision-free 20-photon patterns: their total cannot exceed P_20
    assert prob.sum() <= oracle.photon_number_prob(50, 20, 0.88) * (1 + 1e-12)
    B = oracle.state_B(st_in.U, st_in.r)
    pref = float(np.prod(1.0 / np.cosh(st_in.r)))
    for i in np.linspace(0, len(pats) - 1, 40).astype(int):
        ref = abs(oracle.haf_enum(oracle.pattern_matrix(B, pats[i]))) ** 2 * pref
        assert relerr(prob[i], ref) < TOL, (i, prob[i], ref)


def test_largest_size_block_diagonal(ctx, torch_dev):
    """n = 46 (the largest supported size): Haf of a block-diagonal matrix is the product of the
    blocks' hafnians (no perfect matching crosses the blocks). The blocks are GBS pattern matrices
    B_S of the config-5 state (m = 60, r = 0.88), sizes 24 and 22, built the way
    tests/golden/make_general_golden.py --blockdiag builds them; the exact value is the product of
    the blocks' matching sums. Block-diagonal input is the worst case for the subset sum's
    cancellation (every term mixing the blocks cancels exactly); its kappa (and kappa2), from the
    oracle's double power trace, are stored with it, and the bound is that of tests/bounds.py."""
    path = pathlib.Path(__file__).parent / "golden" / "blockdiag46_haf.json"
    if not path.exists():
        pytest.skip("blockdiag46_haf.json not written yet")
    rec = json.loads(path.read_text())
    rng = np.random.default_rng(46)
    st_in, _ = inputs.config5()
    B = oracle.state_B(st_in.U, st_in.r)
    modes = rng.permutation(60)
    A1 = oracle.pattern_matrix(B, sorted(modes[:24]))
    A2 = oracle.pattern_matrix(B, sorted(modes[24:46]))
    A = np.zeros((46, 46), dtype=np.complex128)
    A[:24, :24] = A1
    A[24:, 24:] = A2
    h = ctx.haf_batch(to_dev(A[None], torch_dev)).cpu().numpy()[0]
    ref = complex(oracle.haf_enum(A1)) * complex(oracle.haf_enum(A2))
    assert ref == complex(*rec["haf_blocks"])
    err = relerr(h, ref)
    b = bounds.bound(46, rec["kappa"], rec.get("kappa2"))  # the reference is exact (block product)
    print(f"n=46 block-diagonal kappa={rec['kappa']:.2e} kappa2={rec.get('kappa2', float('nan')):.2e} "
          f"rel err {err:.2e} bound {b:.2e}")
    assert err <= b
