"""Host-side parameter selection (no GPU): the candidate set, the fixed default
rule and the cost-model features, through the C ABI.  Every candidate must be a
valid product shape (its workspace query succeeds)."""

import math

import pytest

import paper_0810_3203_amd as T


def _shape(len_g, gl, len_h, hl, p):
    bits = 32 * (gl + hl) + (min(len_g, len_h) - 1).bit_length()
    ws = (bits + 31) // 32
    zg, zh = -(-len_g // p.k), -(-len_h // p.k)
    n = zg + zh - 1
    l = max(1, (n - 1).bit_length())
    need = ws if p.k == 1 else (2 * p.k - 1) * ws
    W = 1
    while W < need or 64 * W < (1 << l):
        W *= 2
    return dict(n=n, l=l, W=W, bytes=2 * (1 << l) * (W + 1) * 4)


@pytest.mark.parametrize("lg,gl,lh,hl", [(500, 32, 500, 32), (100, 32, 20000, 32), (20000, 32, 20000, 32),
                                          (1, 1, 1, 1), (7, 2, 3, 2), (3000, 63, 3000, 63)])
def test_candidates_valid_and_ordered(lg, gl, lh, hl):
    cands = T.ss_candidates(lg, gl, lh, hl)
    assert cands and cands[0].k == 1 and cands[0].split.top_l1 == 0
    ks = [c.k for c in cands]
    assert ks == sorted(ks)
    assert len({(c.k, c.split.top_l1, c.pad_rows, c.zeta_exp) for c in cands}) == len(cands)
    for i, c in enumerate(cands):
        if c.zeta_exp:  # follows its untwisted form, with zeta = theta^(3N/2)
            prev = cands[i - 1]
            assert (prev.k, prev.split.top_l1, prev.pad_rows, prev.zeta_exp) == (c.k, c.split.top_l1, c.pad_rows, 0)
            assert c.zeta_exp == 3 * (32 * _shape(lg, gl, lh, hl, c)["W"]) // 2
        elif c.pad_rows:  # follows its unpadded form and that form's twist
            prev = cands[i - 2]
            assert (prev.k, prev.split.top_l1, prev.pad_rows, prev.zeta_exp) == (c.k, c.split.top_l1, 0, 0)
        assert T.zx_mul_ss_workspace(lg, gl, lh, hl, c) == _shape(lg, gl, lh, hl, c)["bytes"]
        if c.split.top_l1:
            assert 1 <= c.split.top_l1 < _shape(lg, gl, lh, hl, c)["l"]


def test_default_rule():
    for lg, lh in [(500, 500), (20000, 20000), (10000, 300), (100, 100)]:
        d = T.ss_default_params(lg, 32, lh, 32)
        fp = {c.k: _shape(lg, 32, lh, 32, c)["bytes"] for c in T.ss_candidates(lg, 32, lh, 32)}
        best = min(fp.values())
        assert d.k == min(k for k, b in fp.items() if 4 * b <= 5 * best)
        assert d.split.top_l1 == 0 and d.N == 0 and d.l == 0


def test_features_finite_and_distinct():
    seen = set()
    for c in T.ss_candidates(12000, 32, 9000, 32):
        f = T.ss_features(12000, 32, 9000, 32, c)
        assert len(f) == T.SS_FEATURES and all(math.isfinite(v) and -1 < v < 4 for v in f)
        seen.add(tuple(round(v, 6) for v in f))
    assert len(seen) == len(T.ss_candidates(12000, 32, 9000, 32))


def test_bad_shapes_rejected():
    with pytest.raises(T.TFTError):
        T.ss_candidates(0, 32, 10, 32)
    with pytest.raises(T.TFTError):
        T.ss_default_params(10, 0, 10, 32)


@pytest.mark.parametrize("lg,lh,N,l,top,leaf,pad", [
    (500, 500, 512, 10, 0, 2, 0), (500, 500, 512, 10, 0, 2, 1), (3000, 2999, 8192, 13, 0, 3, 0),
    (3000, 2999, 8192, 13, 0, 3, 1), (700, 300, 2048, 11, 7, 2, 1), (700, 300, 2048, 11, T.SPLIT_DC, 3, 0),
    (1, 1, 64, 1, 0, 1, 0), (5000, 4000, 16384, 14, 0, 4, 1)])
def test_pass_count_features_match_the_planner(lg, lh, N, l, top, leaf, pad):
    """Features 11 and 13 are the leaf passes of one TFT and of the ITFT, from the
    planner's recursion without building jobs; they must equal the pass counts
    of the schedules the planner builds."""
    p = T.SSParams(N, l, T.Split(top, leaf), 1, pad)
    f = T.ss_features(lg, 1, lh, 1, p)
    n = lg + lh - 1
    l1 = 1 if top == T.SPLIT_DC else (top if 0 < top < l else l // 2)
    L2 = 1 << (l - l1)
    nt = -(-n // L2) * L2 if pad else n
    ring = T.fermat_ring(N)
    pt = max(len(T.Plan(ring, 0, l, 0, z, nt, 0, top, leaf).export()["passes"]) for z in (lg, lh))
    pi = len(T.Plan(ring, 1, l, 0, nt, nt, 0, top, leaf).export()["passes"])
    assert round(f[10] * 8) == pt and round(f[12] * 32) == pi, (f[10] * 8, pt, f[12] * 32, pi)


def test_padding_flag_validated():
    base = T.zx_mul_ss_workspace(300, 4, 200, 4, T.SSParams(0, 0, T.Split(0, 0), 1, 0))
    assert T.zx_mul_ss_workspace(300, 4, 200, 4, T.SSParams(0, 0, T.Split(0, 0), 1, 1)) == base
    with pytest.raises(T.TFTError):
        T.zx_mul_ss_workspace(300, 4, 200, 4, T.SSParams(0, 0, T.Split(0, 0), 1, 2))
