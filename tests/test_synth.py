"""Seeded input generators: SplitMix64 test vector and workload shapes."""

import numpy as np
import pytest

from synth import SplitMix64
from synth import workloads as wl


def test_splitmix64_reference_vector():
    # Published reference outputs of SplitMix64 for seed 1234567.
    g = SplitMix64(1234567)
    assert [g.next() for _ in range(3)] == [6457827717110365317, 3203168211198807973, 9817491932198370423]
    g = SplitMix64(1234567)
    assert [int(v) for v in g.take(3)] == [6457827717110365317, 3203168211198807973, 9817491932198370423]


def test_take_continues_stream():
    a = SplitMix64(5)
    first = [a.next() for _ in range(10)]
    b = SplitMix64(5)
    assert [int(v) for v in b.take(4)] + [int(v) for v in b.take(6)] == first


def test_case_shapes_small():
    g, h = wl.zx_operands(1)
    assert g.shape == (500, 2) and h.shape == (500, 2)
    g, h = wl.zx_operands(2, len_g=10, len_h=7)
    assert g.shape == (10, 63) and h.shape == (7, 63)
    assert int(g[:, 62].max()) < (1 << 16)  # 2000 bits = 62 limbs + 16 bits
    m, g4, h4 = wl.zmx_operands(len_g=1000, len_h=500)
    assert m % 2 == 1 and (1 << 61) <= m < (1 << 62)
    assert g4.shape == (1000,) and int(g4.max()) < m and int(h4.max()) < m


def test_rejection_draw_is_prefix_stable():
    m, g, _ = wl.zmx_operands(len_g=200, len_h=1)
    m2, g2, _ = wl.zmx_operands(len_g=500, len_h=1)
    assert m == m2 and np.array_equal(g, g2[:200])


def test_limb_roundtrip():
    vals = [0, 1, (1 << 100) - 1, 12345678901234567890]
    assert wl.limbs_to_ints(wl.ints_to_limbs(vals, 4)) == vals


def test_batch_lengths_in_range():
    for lg, lh in wl.batch_lengths(64):
        assert 100 <= lg <= 20000 and 100 <= lh <= 20000
    g, h = wl.batch_request(3)
    assert (g.shape[0], h.shape[0]) == wl.batch_lengths(4)[3]
    assert g.shape[1] == 32 and int(g[:, 31].max()) < (1 << 8)


def test_device_generator_matches_numpy():
    torch = pytest.importorskip("torch")
    from synth import device as dev
    from synth.splitmix import SplitMix64
    s = SplitMix64(1234567)
    ref = s.take(1000)
    got = dev.draws(torch, 1234567, 0, 1000, "cpu").numpy().view(np.uint64)
    assert np.array_equal(got, ref)
    for i in (0, 5):
        g, h = wl.batch_request(i, len_lo=10, len_hi=300)
        dg, dh = dev.batch_request(torch, i, "cpu", len_lo=10, len_hi=300)
        assert np.array_equal(dg.numpy().view(np.uint32), g)
        assert np.array_equal(dh.numpy().view(np.uint32), h)
    for bits in (32, 64, 96, 1000):
        s = SplitMix64(99)
        s.take(3)
        ref = wl.random_ints(s, 17, bits)
        got = dev.ints(torch, 99, 3, 17, bits, "cpu").numpy().view(np.uint32)
        assert np.array_equal(got, ref), bits
