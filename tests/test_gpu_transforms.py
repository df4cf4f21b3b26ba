"""GPU parity of the transforms and pointwise products against the oracle.

Every call goes through the C ABI (paper_0810_3203_amd binding of libtft.so).
Outputs must equal the oracle exactly (the work is integer arithmetic).
Inputs carry boundary residues (0, 1, 2^N, 2^N - 1, long runs of ones) and
cells at or beyond z hold random garbage that must never be read.
"""

import random

import numpy as np
import pytest

from oracle import tft_oracle as O
from tests.gpu_util import (fermat_from_device, fermat_to_device, fermat_values, nega_from_device, nega_to_device,
                            note)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0810_3203_amd as T  # noqa: E402


def _fermat_inputs(ring, count, rng):
    p = ring.p
    N = ring.N
    out = []
    for i in range(count):
        k = rng.randrange(10)
        if k == 0:
            out.append(0)
        elif k == 1:
            out.append(p - 1)                 # 2^N
        elif k == 2:
            out.append((1 << N) - 1)          # all ones
        elif k == 3:
            out.append(1)
        elif k == 4:
            out.append(((1 << (N // 2)) - 1) << (N // 4))
        else:
            out.append(rng.randrange(p))
    return out


def _run_tft(N, l, s, z, n, seed, top_l1=0, leaf_log2=0):
    ring = O.FermatRing(N)
    rng = random.Random(seed)
    L = 1 << l
    a = _fermat_inputs(ring, L, rng)  # the tail beyond z is garbage
    note("tft N=%d l=%d s=%d z=%d n=%d split=%d/%d seed=%d" % (N, l, s, z, n, top_l1, leaf_log2, seed))
    x = fermat_to_device(a, N, L, torch)
    if top_l1 or leaf_log2:
        T.Plan(T.fermat_ring(N), 0, l, s, z, n, 0, top_l1, leaf_log2).execute(x)
    else:
        T.tft_forward(T.fermat_ring(N), l, s, z, n, x)
    torch.cuda.synchronize()
    got = fermat_values(*fermat_from_device(x, N, L, n))
    assert got == O.tft(ring, L, s, z, n, a[:z]), (N, l, s, z, n)


def _run_itft(N, l, s, z, n, f, seed, top_l1=0, leaf_log2=0):
    ring = O.FermatRing(N)
    rng = random.Random(seed)
    L = 1 << l
    a = _fermat_inputs(ring, z, rng)
    inputs, expect = O.itft_case(ring, L, s, z, n, f, a)
    cells = list(inputs) + _fermat_inputs(ring, L - z, rng)
    note("itft N=%d l=%d s=%d z=%d n=%d f=%d split=%d/%d seed=%d" % (N, l, s, z, n, f, top_l1, leaf_log2, seed))
    x = fermat_to_device(cells, N, L, torch)
    if top_l1 or leaf_log2:
        T.Plan(T.fermat_ring(N), 1, l, s, z, n, f, top_l1, leaf_log2).execute(x)
    else:
        T.itft_inverse(T.fermat_ring(N), l, s, z, n, f, x)
    torch.cuda.synchronize()
    got = fermat_values(*fermat_from_device(x, N, L, n + f))
    assert got == expect, (N, l, s, z, n, f)


SMALL_RINGS = [32, 64, 128, 256, 512, 1024, 2048, 4096, 8192]


@pytest.mark.parametrize("N", SMALL_RINGS)
def test_tft_single_leaf(N):
    rng = random.Random(N)
    for l in (1, 2, 3, 5):
        L = 1 << l
        for z, n in {(1, 1), (L, L), (1, L), (L, 1), (rng.randint(1, L), rng.randint(1, L))}:
            _run_tft(N, l, rng.randrange(2 * N), z, n, seed=N + 7 * z + n)


@pytest.mark.parametrize("N", SMALL_RINGS)
def test_itft_single_leaf(N):
    rng = random.Random(N + 1)
    for l in (1, 2, 3, 5):
        L = 1 << l
        cases = {(L, L, 0), (1, 1, 0), (1, 0, 1), (L, L - 1, 1), (L, 0, 1)}
        z = rng.randint(1, L)
        nn = rng.randint(0, z)
        cases.add((z, nn, 1 if nn < L else 0) if nn else (z, 0, 1))
        for z, n, f in cases:
            _run_itft(N, l, rng.randrange(2 * N), z, n, f, seed=N + 3 * z + n)


@pytest.mark.parametrize("N,leaf", [(64, 1), (64, 2), (512, 3), (4096, 2), (65536, 2), (65536, 3)])
def test_tft_multipass(N, leaf):
    rng = random.Random(N * leaf)
    for l in (4, 6):
        L = 1 << l
        for z, n in {(L, L), (rng.randint(1, L), rng.randint(1, L)), (3, L - 1)}:
            _run_tft(N, l, rng.randrange(2 * N), z, n, seed=z + n, leaf_log2=leaf)


@pytest.mark.parametrize("N,leaf", [(64, 1), (64, 2), (512, 3), (4096, 2), (65536, 2), (65536, 3)])
def test_itft_multipass(N, leaf):
    rng = random.Random(N * leaf + 1)
    for l in (4, 6):
        L = 1 << l
        for z, n, f in {(L, L, 0), (L - 3, L - 5, 1), (rng.randint(L // 2, L), rng.randint(1, L // 2), 0)}:
            _run_itft(N, l, rng.randrange(2 * N), z, n, f, seed=z + n, leaf_log2=leaf)


@pytest.mark.parametrize("N", [32, 64, 512, 2048, 65536])
def test_shift_edges(N):
    """Length-2 transforms multiply one cell by theta^s directly: every shift class
    (0, 1, 31, 32, N-1, N, 2N-1) on all-ones, 2^N, 0 and 1 operands."""
    ring = O.FermatRing(N)
    ones, top = (1 << N) - 1, ring.p - 1
    rng = random.Random(N + 5)
    pairs = [(ones, ones), (top, 1), (0, top), (top, top), (rng.randrange(ring.p), ones), (1, ones)]
    for s in sorted({0, 1, 31, 32, N - 1, N, 2 * N - 1}):
        note("shift edges N=%d s=%d" % (N, s))
        for a0, a1 in pairs:
            x = fermat_to_device([a0, a1], N, 2, torch)
            T.tft_forward(T.fermat_ring(N), 1, s, 2, 2, x)
            torch.cuda.synchronize()
            assert fermat_values(*fermat_from_device(x, N, 2, 2)) == O.tft(ring, 2, s, 2, 2, [a0, a1]), (s, a0, a1)
            inputs, expect = O.itft_case(ring, 2, s, 2, 2, 0, [a0, a1])
            y = fermat_to_device(list(inputs), N, 2, torch)
            T.itft_inverse(T.fermat_ring(N), 1, s, 2, 2, 0, y)
            torch.cuda.synchronize()
            assert fermat_values(*fermat_from_device(y, N, 2, 2)) == expect, (s, a0, a1)


LARGE_RINGS = [16384, 32768, 131072]  # 512, 1024 and 4096 limbs a cell


@pytest.mark.parametrize("N", LARGE_RINGS)
def test_tft_large_rings(N):
    rng = random.Random(N + 11)
    for l, leaf in ((3, 0), (5, 0), (5, 2)):
        L = 1 << l
        for z, n in {(L, L), (1, L), (rng.randint(2, L), rng.randint(1, L))}:
            _run_tft(N, l, rng.randrange(2 * N), z, n, seed=N + z + 5 * n, leaf_log2=leaf)


@pytest.mark.parametrize("N", LARGE_RINGS)
def test_itft_large_rings(N):
    rng = random.Random(N + 12)
    for l, leaf in ((3, 0), (5, 0), (5, 2)):
        L = 1 << l
        for z, n, f in {(L, L, 0), (L, L - 1, 1), (L - 3, rng.randint(1, L - 4), 1)}:
            _run_itft(N, l, rng.randrange(2 * N), z, n, f, seed=N + z + 3 * n, leaf_log2=leaf)


def test_divide_and_conquer_split_on_gpu():
    rng = random.Random(91)
    for N, l, leaf in ((512, 6, 2), (512, 8, 3), (8192, 7, 1)):
        L = 1 << l
        for z, n in {(L, L), (L // 2 + 3, L - 5), (rng.randint(1, L), rng.randint(1, L))}:
            _run_tft(N, l, rng.randrange(2 * N), z, n, seed=z + n, top_l1=T.SPLIT_DC, leaf_log2=leaf)
        for z, n, f in {(L, L, 0), (L - 3, L - 7, 1), (L // 2, L // 4 + 1, 0)}:
            _run_itft(N, l, rng.randrange(2 * N), z, n, f, seed=z + n, top_l1=T.SPLIT_DC, leaf_log2=leaf)


def test_every_top_split_on_gpu():
    for top in (1, 2, 3, 4, 5):
        _run_tft(512, 6, 77, 40, 61, seed=top, top_l1=top, leaf_log2=2)
        _run_itft(512, 6, 77, 50, 43, 1, seed=top, top_l1=top, leaf_log2=2)


@pytest.mark.parametrize("N", [32, 64, 512, 4096, 16384, 32768, 65536, 131072])
def test_pointwise(N):
    ring = O.FermatRing(N)
    rng = random.Random(N)
    cap, n = 40, 37
    a = _fermat_inputs(ring, cap, rng)
    b = _fermat_inputs(ring, cap, rng)
    a[0], b[0] = ring.p - 1, ring.p - 1  # (2^N)(2^N)
    a[1], b[2] = ring.p - 1, ring.p - 1
    for scale in (0, 1, 7, 17):
        note("pointwise N=%d n=%d scale=%d" % (N, n, scale))
        da, db = fermat_to_device(a, N, cap, torch), fermat_to_device(b, N, cap, torch)
        dc = torch.zeros_like(da)
        T.pointwise_mul(T.fermat_ring(N), n, da, db, dc, cap, scale)
        T.pointwise_mul(T.fermat_ring(N), n, da, db, da, cap, scale)  # in place
        torch.cuda.synchronize()
        expect = O.pointwise(ring, a[:n], b[:n], scale)
        assert fermat_values(*fermat_from_device(dc, N, cap, n)) == expect
        assert fermat_values(*fermat_from_device(da, N, cap, n)) == expect


@pytest.mark.parametrize("N", [16384, 32768, 65536, 131072])
def test_pointwise_nested_extremes(N):
    """The sizes whose products take one more Schoenhage-Strassen level (64
    pieces, inner transforms over Z/(2^N'+1)): operands that make every piece
    and every inner coefficient as large as it gets, single pieces at either
    end, runs of all-ones limbs, 0, 1, 2^N - 1, and 2^N, with and without a
    scale factor, against the oracle's product."""
    ring = O.FermatRing(N)
    rng = random.Random(N + 1)
    top = (1 << N) - 1
    piece = 1 << (N // 64)
    a = [top, top, 0, 1, piece - 1, (piece - 1) << (N - N // 64), 1 << (N - 1), ring.p - 1, top]
    b = [top, rng.getrandbits(N), rng.getrandbits(N), rng.getrandbits(N), (piece - 1) << (N - N // 64),
         (piece - 1) << (N - N // 64), 1 << (N - 1), top, ring.p - 1]
    for _ in range(3):
        v = 0
        for q in range(N // 32):
            v |= (0xFFFFFFFF if rng.random() < 0.5 else 0) << (32 * q)
        a.append(v)
        b.append(rng.getrandbits(N))
    n = cap = len(a)
    for scale in (0, 5):
        note("pointwise nested extremes N=%d scale=%d" % (N, scale))
        da, db = fermat_to_device(a, N, cap, torch), fermat_to_device(b, N, cap, torch)
        dc = torch.zeros_like(da)
        T.pointwise_mul(T.fermat_ring(N), n, da, db, dc, cap, scale)
        torch.cuda.synchronize()
        assert fermat_values(*fermat_from_device(dc, N, cap, n)) == O.pointwise(ring, a, b, scale)


# ---------------------------------------------------------------------------
# (Z/mZ)[y]/(y^K+1)
# ---------------------------------------------------------------------------

def _nega_inputs(ring, count, rng):
    out = []
    for _ in range(count):
        k = rng.randrange(6)
        if k == 0:
            out.append(ring.zero())
        elif k == 1:
            out.append(tuple([ring.m - 1] * ring.K))
        else:
            out.append(tuple(rng.randrange(ring.m) for _ in range(ring.K)))
    return out


@pytest.mark.parametrize("K", [2, 16, 64, 256, 1024])
def test_nega_transforms(K):
    rng = random.Random(K)
    m = (rng.getrandbits(62) | (1 << 61) | 1) & ((1 << 62) - 1)
    ring = O.NegaRing(K, m)
    for l, leaf in [(1, 0), (3, 0), (4, 2), (5, 0)]:
        L = 1 << l
        if 2 * K % L:
            continue
        for z, n in {(L, L), (rng.randint(1, L), rng.randint(1, L))}:
            a = _nega_inputs(ring, L, rng)
            s = rng.randrange(2 * K)
            note("nega tft K=%d l=%d z=%d n=%d s=%d" % (K, l, z, n, s))
            x = nega_to_device(a, K, L, torch)
            T.Plan(T.nega_ring(K, m), 0, l, s, z, n, 0, 0, leaf).execute(x)
            torch.cuda.synchronize()
            assert nega_from_device(x, K, n) == O.tft(ring, L, s, z, n, a[:z])
        for z, n, f in {(L, L, 0), (L, L - 1, 1), (rng.randint(1, L), 0, 1)}:
            a = _nega_inputs(ring, z, rng)
            s = rng.randrange(2 * K)
            inputs, expect = O.itft_case(ring, L, s, z, n, f, a)
            note("nega itft K=%d l=%d z=%d n=%d f=%d s=%d" % (K, l, z, n, f, s))
            x = nega_to_device(list(inputs) + _nega_inputs(ring, L - z, rng), K, L, torch)
            T.Plan(T.nega_ring(K, m), 1, l, s, z, n, f, 0, leaf).execute(x)
            torch.cuda.synchronize()
            assert nega_from_device(x, K, n + f) == expect


def test_nega_divide_and_conquer_split():
    K = 64
    rng = random.Random(641)
    m = (rng.getrandbits(62) | (1 << 61) | 1) & ((1 << 62) - 1)
    ring = O.NegaRing(K, m)
    for l, leaf in [(5, 2), (7, 1)]:
        L = 1 << l
        for z, n in {(L, L), (L - 5, L // 2 + 1)}:
            a = _nega_inputs(ring, L, rng)
            s = rng.randrange(2 * K)
            note("nega tft divide-and-conquer K=%d l=%d z=%d n=%d s=%d leaf=%d" % (K, l, z, n, s, leaf))
            x = nega_to_device(a, K, L, torch)
            T.Plan(T.nega_ring(K, m), 0, l, s, z, n, 0, T.SPLIT_DC, leaf).execute(x)
            torch.cuda.synchronize()
            assert nega_from_device(x, K, n) == O.tft(ring, L, s, z, n, a[:z])
        for z, n, f in {(L, L, 0), (L - 2, L - 9, 1)}:
            a = _nega_inputs(ring, z, rng)
            s = rng.randrange(2 * K)
            inputs, expect = O.itft_case(ring, L, s, z, n, f, a)
            note("nega itft divide-and-conquer K=%d l=%d z=%d n=%d f=%d s=%d leaf=%d" % (K, l, z, n, f, s, leaf))
            x = nega_to_device(list(inputs) + _nega_inputs(ring, L - z, rng), K, L, torch)
            T.Plan(T.nega_ring(K, m), 1, l, s, z, n, f, T.SPLIT_DC, leaf).execute(x)
            torch.cuda.synchronize()
            assert nega_from_device(x, K, n + f) == expect


@pytest.mark.parametrize("K", [2, 1024, 4096])
def test_nega_pointwise_extreme_values(K):
    """Coefficients m - 1 and 0 (a zero entering the negated wrap is m), 62-bit modulus."""
    m = (1 << 62) - 57
    ring = O.NegaRing(K, m)
    a = [[m - 1] * K, [m - 1 if j % 3 else 0 for j in range(K)], [0] * K]
    b = [[0 if j % 2 else m - 1 for j in range(K)], [m - 1] * K, [m - 1] * K]
    note("nega pointwise extreme values K=%d" % K)
    da, db = nega_to_device(a, K, 3, torch), nega_to_device(b, K, 3, torch)
    dc = torch.zeros_like(da)
    T.pointwise_mul(T.nega_ring(K, m), 3, da, db, dc, 3, 5)
    torch.cuda.synchronize()
    assert nega_from_device(dc, K, 3) == O.pointwise(ring, a, b, 5)


@pytest.mark.parametrize("K", [2, 16, 64, 1024])
def test_nega_pointwise(K):
    rng = random.Random(K + 5)
    for m in ((1 << 62) - 57, 3, 1000003):
        ring = O.NegaRing(K, m)
        cap, n = (6, 5) if K <= 64 else (3, 2)
        a = _nega_inputs(ring, cap, rng)
        b = _nega_inputs(ring, cap, rng)
        for scale in (0, 3, 11):
            note("nega pointwise K=%d m=%d scale=%d" % (K, m, scale))
            da, db = nega_to_device(a, K, cap, torch), nega_to_device(b, K, cap, torch)
            dc = torch.zeros_like(da)
            T.pointwise_mul(T.nega_ring(K, m), n, da, db, dc, cap, scale)
            torch.cuda.synchronize()
            assert nega_from_device(dc, K, n) == O.pointwise(ring, a[:n], b[:n], scale)


def _times_pow2_mod(a, k, m):
    """a * 2^k mod m for uint64 arrays with entries < m < 2^62 (repeated doubling, no overflow)."""
    a = np.array(a, dtype=np.uint64)
    mm = np.uint64(m)
    for _ in range(k):
        a = a * np.uint64(2)
        a = np.where(a >= mm, a - mm, a)
    return a


@pytest.mark.parametrize("s", [0, 1537])
def test_nega_transforms_case4_shape(coracle, s):
    """TFT and ITFT at the shape of the Schoenhage-Nussbaumer product (Sect. 5.2):
    K = 1024, L = 2^11 (several leaf passes), z = 977 pieces, n = 1953, the
    product's 62-bit modulus.  Every TFT output is compared with eq. (1) in the C
    oracle; the ITFT is checked by construction for (z, n, f) = (n, n, 0), the
    product's inverse, and (n, n - 1, 1)."""
    from synth import workloads as wl
    m = wl.zmx_operands(len_g=1, len_h=1)[0]
    K, l, z, n = 1024, 11, 977, 1953
    L = 1 << l
    rng = np.random.default_rng(4 + s)
    a = (rng.integers(0, 1 << 62, size=(L, K), dtype=np.uint64) % np.uint64(m)).astype(np.uint64)
    a[0] = m - 1
    a[1, ::2] = 0
    ring = T.nega_ring(K, m)
    note("nega tft K=%d l=%d z=%d n=%d s=%d (product shape)" % (K, l, z, n, s))
    x = torch.from_numpy(a.reshape(-1).view(np.int64)).cuda()
    T.tft_forward(ring, l, s, z, n, x)
    torch.cuda.synchronize()
    got = x.cpu().numpy().view(np.uint64).reshape(L, K)[:n]
    expect = coracle.nega_dft_sampled(K, m, L, s, a[:z], list(range(n)))
    bad = np.nonzero(np.any(got != expect, axis=1))[0]
    assert len(bad) == 0, "TFT outputs differ at %s" % bad[:8].tolist()

    b = (rng.integers(0, 1 << 62, size=(n, K), dtype=np.uint64) % np.uint64(m)).astype(np.uint64)
    ahat = coracle.nega_dft_sampled(K, m, L, s, b, list(range(n)))
    Lb = _times_pow2_mod(b, l, m)
    for zz, nn, f in ((n, n, 0), (n, n - 1, 1)):
        note("nega itft K=%d l=%d z=%d n=%d f=%d s=%d (product shape)" % (K, l, zz, nn, f, s))
        fill = (rng.integers(0, 1 << 62, size=(L, K), dtype=np.uint64) % np.uint64(m)).astype(np.uint64)
        fill[:nn] = ahat[:nn]
        fill[nn:zz] = Lb[nn:zz]
        x = torch.from_numpy(fill.reshape(-1).view(np.int64)).cuda()
        T.itft_inverse(ring, l, s, zz, nn, f, x)
        torch.cuda.synchronize()
        got = x.cpu().numpy().view(np.uint64).reshape(L, K)
        bad = np.nonzero(np.any(got[:nn] != Lb[:nn], axis=1))[0]
        assert len(bad) == 0, "ITFT outputs differ at %s" % bad[:8].tolist()
        if f:
            assert np.array_equal(got[nn], ahat[nn]), "ITFT f output differs"
