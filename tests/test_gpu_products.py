"""GPU parity of the two products (Sect. 5) against the schoolbook oracle.

Z[x] by Schoenhage-Strassen (zx_mul_ss) and (Z/mZ)[x] by Schoenhage-Nussbaumer
(zmx_mul_nussbaumer), through the C ABI.  Small shapes are compared in full;
the benchmark shapes are compared on sampled coefficients the oracle computes
one by one, plus (for Z[x]) Schwartz-Zippel fingerprints of the whole output:
sum_k u_k r^k = g(r) h(r) mod P for two primes P.
"""

import random

import numpy as np
import pytest

from synth import workloads as wl
from tests.gpu_util import note, u32_to_device, u64_to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0810_3203_amd as T  # noqa: E402

PRIMES = [(1 << 61) - 1, (1 << 62) - 57]


def _out_limbs(g, h):
    bits = 32 * (g.shape[1] + h.shape[1]) + max(0, (min(g.shape[0], h.shape[0]) - 1).bit_length())
    return (bits + 31) // 32


def _zx_gpu(g, h, params=None):
    ow = _out_limbs(g, h)
    out = torch.zeros((g.shape[0] + h.shape[0] - 1, ow), dtype=torch.int32, device="cuda")
    T.zx_mul_ss(u32_to_device(g, torch), u32_to_device(h, torch), out, params)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32), ow


def _check_sampled(coracle, g, h, got, ow, ks):
    ks = sorted(set(int(k) for k in ks))
    expect = coracle.zx_coeffs(g, h, ks, ow)
    assert np.array_equal(got[ks], expect), "sampled coefficients differ"


def _check_fingerprint(coracle, g, h, got, seed):
    rng = random.Random(seed)
    for P in PRIMES:
        r = rng.randrange(2, P - 1)
        lhs = coracle.fingerprint(got, P, r)
        rhs = coracle.fingerprint(g, P, r) * coracle.fingerprint(h, P, r) % P
        assert lhs == rhs, "fingerprint mod %d differs" % P


@pytest.mark.parametrize("lg,lh,bits", [(1, 1, 64), (1, 7, 32), (13, 5, 64), (100, 37, 96), (257, 300, 64)])
def test_zx_small_full(coracle, lg, lh, bits):
    gen = random.Random(lg * 1000 + lh)
    from synth.splitmix import SplitMix64
    s = SplitMix64(gen.getrandbits(64))
    g, h = wl.random_ints(s, lg, bits), wl.random_ints(s, lh, bits)
    g[0] = 0xFFFFFFFF  # all-ones coefficients push the largest carries
    h[-1] = 0xFFFFFFFF
    note("zx_mul_ss small %d x %d, %d bits" % (lg, lh, bits))
    got, ow = _zx_gpu(g, h)
    _check_sampled(coracle, g, h, got, ow, range(lg + lh - 1))


def test_zx_explicit_ring_and_splits(coracle):
    from synth.splitmix import SplitMix64
    s = SplitMix64(77)
    g, h = wl.random_ints(s, 60, 64), wl.random_ints(s, 70, 64)
    for N, l, top, leaf in [(1024, 8, 0, 0), (2048, 9, 3, 2), (512, 8, 1, 3), (8192, 8, 5, 1)]:
        note("zx_mul_ss explicit N=%d l=%d split %d/%d" % (N, l, top, leaf))
        got, ow = _zx_gpu(g, h, T.SSParams(N, l, T.Split(top, leaf)))
        _check_sampled(coracle, g, h, got, ow, range(129))


def test_zx_divide_and_conquer_split(coracle):
    """L1 = 2 at every level above the leaf gives the same product (Sect. 1)."""
    from synth.splitmix import SplitMix64
    s = SplitMix64(78)
    g, h = wl.random_ints(s, 700, 250), wl.random_ints(s, 450, 250)
    for N, l, leaf in [(0, 0, 0), (1024, 11, 3), (2048, 11, 1)]:
        note("zx_mul_ss divide-and-conquer split N=%d l=%d leaf=%d" % (N, l, leaf))
        got, ow = _zx_gpu(g, h, T.SSParams(N, l, T.Split(T.SPLIT_DC, leaf)))
        _check_sampled(coracle, g, h, got, ow, range(1149))


def test_zx_whole_row_padding(coracle):
    """n rounded up to whole rows of the top split (Sect. 6) gives the same product."""
    from synth.splitmix import SplitMix64
    s = SplitMix64(79)
    g, h = wl.random_ints(s, 611, 300), wl.random_ints(s, 390, 300)
    for p in [T.SSParams(0, 0, T.Split(0, 0), 1, 1), T.SSParams(0, 0, T.Split(3, 0), 1, 1),
              T.SSParams(0, 0, T.Split(T.SPLIT_DC, 2), 1, 1), T.SSParams(0, 0, T.Split(0, 0), 3, 1),
              T.SSParams(32768, 11, T.Split(0, 2), 1, 1)]:
        note("zx_mul_ss whole rows N=%d l=%d k=%d split %d/%d" % (p.N, p.l, p.k, p.split.top_l1, p.split.leaf_log2))
        got, ow = _zx_gpu(g, h, p)
        _check_sampled(coracle, g, h, got, ow, range(1000))


def test_zx_twisted_transforms(coracle):
    """TFT(g), TFT(h) twisted by zeta = theta^s and the ITFT by zeta^2 give the same product."""
    from synth.splitmix import SplitMix64
    s = SplitMix64(80)
    g, h = wl.random_ints(s, 500, 200), wl.random_ints(s, 433, 200)
    for N, zexp, pad in [(0, 1, 0), (16384, 24576, 0), (16384, 24576, 1), (16384, 32767, 0), (0, 12345, 1),
                         (16384, 1 << 31, 0)]:
        p = T.SSParams(N, 0, T.Split(0, 0), 1, pad, zexp)
        note("zx_mul_ss twist s=%d N=%d pad=%d" % (zexp, N, pad))
        got, ow = _zx_gpu(g, h, p)
        _check_sampled(coracle, g, h, got, ow, range(932))


def test_zx_case1_full(coracle):
    g, h = wl.zx_operands(1)
    note("zx_mul_ss case 1 (500 x 500, 64-bit)")
    got, ow = _zx_gpu(g, h)
    _check_sampled(coracle, g, h, got, ow, range(999))


def test_zx_case2_full_size(coracle):
    g, h = wl.zx_operands(2)
    note("zx_mul_ss case 2 (3000 x 3000, 2000-bit)")
    got, ow = _zx_gpu(g, h)
    rng = random.Random(2)
    ks = list(range(8)) + list(range(5991, 5999)) + [rng.randrange(5999) for _ in range(24)]
    _check_sampled(coracle, g, h, got, ow, ks)
    _check_fingerprint(coracle, g, h, got, 2)


def test_zx_case3_full_size(coracle):
    g, h = wl.zx_operands(3)
    note("zx_mul_ss case 3 (50000 x 50000, 32000-bit)")
    got, ow = _zx_gpu(g, h)
    assert got.shape == (99999, 2001)
    ks = list(range(6)) + list(range(99993, 99999)) + [700, 99999 - 701]
    _check_sampled(coracle, g, h, got, ow, ks)
    _check_fingerprint(coracle, g, h, got, 3)


# ---------------------------------------------------------------------------
# Schoenhage-Nussbaumer
# ---------------------------------------------------------------------------

def _zmx_gpu(g, h, m, log2K):
    out = torch.zeros(len(g) + len(h) - 1, dtype=torch.int64, device="cuda")
    T.zmx_mul_nussbaumer(u64_to_device(g, torch), u64_to_device(h, torch), m, log2K, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("lg,lh,log2K,m", [(1, 1, 1, 3), (5, 9, 3, 1000003), (300, 200, 5, (1 << 62) - 57),
                                           (3000, 2000, 7, (1 << 61) + 1), (1024, 1024, 10, 12345677),
                                           (5000, 3000, 11, (1 << 62) - 57), (6000, 9000, 12, (1 << 62) - 57)])
def test_zmx_small_full(coracle, lg, lh, log2K, m):
    rng = np.random.default_rng(lg + lh)
    g = (rng.integers(0, 1 << 62, size=lg, dtype=np.uint64) % np.uint64(m)).astype(np.uint64)
    h = (rng.integers(0, 1 << 62, size=lh, dtype=np.uint64) % np.uint64(m)).astype(np.uint64)
    g[0] = m - 1
    h[-1] = m - 1
    note("zmx_mul_nussbaumer %d x %d K=2^%d m=%d" % (lg, lh, log2K, m))
    got = _zmx_gpu(g, h, m, log2K)
    expect = coracle.zmx_coeffs(g, h, m, list(range(lg + lh - 1)))
    assert np.array_equal(got, expect)


def test_zmx_case4_full_size(coracle):
    """The 500,000 x 500,000 product (K = 1024, 977 pieces of 512 per operand).

    Whole output: sum_k u_k r^k = g(r) h(r) (mod m) at two random points r; the
    identity holds in Z/mZ for the product reduced coefficient by coefficient, so
    a wrong piece (about 1024 outputs) changes the sum unless r is a root of the
    error polynomial.  Coefficients: every piece boundary 512k - 1, 512k, 512k + 1
    (the overlap-add of Sect. 5.2 joins pieces there), the ends, and random ones,
    each by its schoolbook sum."""
    m, g, h = wl.zmx_operands()
    note("zmx_mul_nussbaumer case 4 (500000 x 500000, K = 1024)")
    got = _zmx_gpu(g, h, m, 10)
    assert got.shape == (999999,)
    assert int(got.max()) < m
    rng = random.Random(4)
    for _ in range(2):
        r = rng.randrange(2, m - 1)
        lhs = coracle.fingerprint64(got, m, r)
        rhs = coracle.fingerprint64(g, m, r) * coracle.fingerprint64(h, m, r) % m
        assert lhs == rhs, "fingerprint mod m differs"
    ks = list(range(4)) + list(range(999995, 999999)) + [rng.randrange(999999) for _ in range(120)]
    ks += [512 * k + d for k in range(1, 1954) for d in (-1, 0, 1) if 0 <= 512 * k + d < 999999]
    ks = sorted(set(ks))
    expect = coracle.zmx_coeffs(g, h, m, ks)
    bad = [k for k, e in zip(ks, expect) if int(got[k]) != int(e)]
    assert not bad, "coefficients differ at %s" % bad[:8]
