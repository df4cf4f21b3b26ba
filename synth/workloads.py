"""Seeded synthetic workloads with the shapes of the five benchmark cases.

Every workload draws from SplitMix64 with seed ``SEED_BASE + c`` for case c.
A b-bit value is ceil(b/64) consecutive draws, little-endian, masked to b bits.
Operand g is drawn before operand h.  Values are returned as little-endian
uint32 limb arrays of shape (count, ceil(b/32)); ``limbs_to_ints`` and
``ints_to_limbs`` convert between that layout and Python integers.

Cases (sizes follow the workloads of the paper's Sect. 5 experiments):
  1: Z[x], 500 x 500 coefficients of 64 bits   (ring Z/(2^512+1),   L = 2^10)
  2: Z[x], 3000 x 3000 coefficients of 2000 bits (ring Z/(2^4096+1), L = 2^13)
  3: Z[x], 50000 x 50000 coefficients of 32000 bits (Z/(2^65536+1), L = 2^17)
  4: (Z/mZ)[x], 500000 x 500000 coefficients, m a random odd 62-bit modulus
  5: 4096 independent Z[x] products, lengths uniform in [100, 20000],
     1000-bit coefficients
"""

import numpy as np

from .splitmix import SplitMix64

SEED_BASE = 0x0810320300000000


def case_seed(c: int) -> int:
    return SEED_BASE + int(c)


# ---------------------------------------------------------------------------
# layout helpers (no arithmetic of the method: only packing of bits)
# ---------------------------------------------------------------------------

def limbs32(bits: int) -> int:
    return (int(bits) + 31) // 32


def draws_to_limbs(draws: np.ndarray, bits: int) -> np.ndarray:
    """(count, d) uint64 draws -> (count, ceil(bits/32)) uint32, masked to ``bits``."""
    count = draws.shape[0]
    w = limbs32(bits)
    u32 = np.ascontiguousarray(draws, dtype=np.uint64).view(np.uint32).reshape(count, -1)
    out = np.array(u32[:, :w], dtype=np.uint32, copy=True)
    rem = bits - 32 * (w - 1)
    if rem < 32:
        out[:, w - 1] &= np.uint32((1 << rem) - 1)
    return out


def random_ints(gen: SplitMix64, count: int, bits: int) -> np.ndarray:
    d = (int(bits) + 63) // 64
    return draws_to_limbs(gen.take(count * d).reshape(count, d), bits)


def limbs_to_ints(limbs: np.ndarray) -> list:
    """uint32 limb rows -> list of Python ints (little-endian limbs)."""
    limbs = np.ascontiguousarray(limbs, dtype=np.uint32)
    if limbs.ndim == 1:
        limbs = limbs.reshape(1, -1)
    return [int.from_bytes(row.tobytes(), "little") for row in limbs]


def ints_to_limbs(values, w: int) -> np.ndarray:
    """Python ints (each < 2^(32w)) -> (count, w) uint32 limb rows."""
    values = list(values)
    out = np.zeros((len(values), w), dtype=np.uint32)
    for i, v in enumerate(values):
        v = int(v)
        if v < 0 or v.bit_length() > 32 * w:
            raise ValueError("value does not fit in %d limbs" % w)
        out[i] = np.frombuffer(v.to_bytes(4 * w, "little"), dtype=np.uint32)
    return out


# ---------------------------------------------------------------------------
# benchmark cases
# ---------------------------------------------------------------------------

ZX_CASES = {
    1: dict(len_g=500, len_h=500, bits=64, N=512, l=10),
    2: dict(len_g=3000, len_h=3000, bits=2000, N=4096, l=13),
    3: dict(len_g=50000, len_h=50000, bits=32000, N=65536, l=17),
}


def zx_operands(c: int, len_g=None, len_h=None):
    """Operands (g, h) of Z[x] case c as uint32 limb arrays.

    ``len_g``/``len_h`` cut the draw short (the first coefficients of the full
    case, for reduced-size tests); they do not change the values drawn.
    """
    spec = ZX_CASES[c]
    gen = SplitMix64(case_seed(c))
    bits = spec["bits"]
    d = (bits + 63) // 64
    lg = spec["len_g"] if len_g is None else int(len_g)
    lh = spec["len_h"] if len_h is None else int(len_h)
    g = random_ints(gen, spec["len_g"], bits)[:lg]
    h = random_ints(gen, spec["len_h"], bits)[:lh]
    del d
    return g, h


ZMX_CASE4 = dict(len_g=500000, len_h=500000, K=1024, l=11)


def _draw_below(gen: SplitMix64, m: int, count: int) -> np.ndarray:
    """``count`` values d >> 2 (in draw order) with rejection of those >= m."""
    out = np.empty(count, dtype=np.uint64)
    have = 0
    mm = np.uint64(m)
    while have < count:
        need = count - have
        block = gen.take(need + need // 2 + 16) >> np.uint64(2)
        acc = block[block < mm]
        take = min(len(acc), need)
        out[have:have + take] = acc[:take]
        have += take
        if take < len(acc):
            # rewind the generator to just after the last draw used
            used = int(np.nonzero(block < mm)[0][take - 1]) + 1
            gen.count -= len(block) - used
    return out


def zmx_operands(len_g=None, len_h=None, seed=None):
    """Case 4: (m, g, h), m odd in [2^61, 2^62), coefficients uniform in [0, m)."""
    gen = SplitMix64(case_seed(4) if seed is None else seed)
    d = gen.next()
    m = (d >> 2) | (1 << 61) | 1
    lg = ZMX_CASE4["len_g"] if len_g is None else int(len_g)
    lh = ZMX_CASE4["len_h"] if len_h is None else int(len_h)
    g = _draw_below(gen, m, lg)
    h = _draw_below(gen, m, lh)
    return m, g, h


BATCH_CASE5 = dict(count=4096, len_lo=100, len_hi=20000, bits=1000)


def batch_request(i: int, bits: int = 1000, len_lo: int = 100, len_hi: int = 20000):
    """Request i of case 5: its own SplitMix64 stream, seed case_seed(5) + (i+1)*2^40.

    Draws len_g, len_h (uniform in [len_lo, len_hi], inclusive), then g, then h.
    """
    gen = SplitMix64(case_seed(5) + ((i + 1) << 40))
    span = len_hi - len_lo + 1
    lg = len_lo + gen.next() % span
    lh = len_lo + gen.next() % span
    g = random_ints(gen, lg, bits)
    h = random_ints(gen, lh, bits)
    return g, h


def batch_lengths(count: int = 4096, len_lo: int = 100, len_hi: int = 20000):
    """(len_g, len_h) of the first ``count`` case-5 requests without drawing coefficients."""
    out = []
    span = len_hi - len_lo + 1
    for i in range(count):
        gen = SplitMix64(case_seed(5) + ((i + 1) << 40))
        out.append((len_lo + gen.next() % span, len_lo + gen.next() % span))
    return out


# ---------------------------------------------------------------------------
# generic random cells for transform tests
# ---------------------------------------------------------------------------

def fermat_cells(seed: int, count: int, W: int, edges: bool = True):
    """Random canonical residues mod 2^(32W)+1 as (limbs (count, W) uint32, tops (count,) uint32).

    A residue is limbs + tops * 2^(32W); tops = 1 only with all limbs zero (the
    residue 2^(32W)).  With ``edges`` a share of the cells take boundary
    patterns: 0, 1, 2^(32W), 2^(32W)-1, single high bits and long runs of ones.
    """
    gen = SplitMix64(seed)
    limbs = gen.take(count * W).view(np.uint32)[: count * W].reshape(count, W).copy()
    tops = np.zeros(count, dtype=np.uint32)
    if edges and count:
        pick = gen.take(count) % np.uint64(16)
        for i in range(count):
            k = int(pick[i])
            if k == 0:
                limbs[i] = 0
            elif k == 1:
                limbs[i] = 0
                tops[i] = 1
            elif k == 2:
                limbs[i] = 0xFFFFFFFF
            elif k == 3:
                limbs[i] = 0
                limbs[i, 0] = 1
            elif k == 4:
                limbs[i] = 0
                limbs[i, W - 1] = 0x80000000
            elif k == 5:
                limbs[i, : W // 2 + 1] = 0xFFFFFFFF
            elif k == 6:
                limbs[i, 1:] = 0
    return limbs, tops


def nega_cells(seed: int, count: int, K: int, m: int, edges: bool = True) -> np.ndarray:
    """Random elements of (Z/mZ)[y]/(y^K+1) as (count, K) uint64 coefficient rows in [0, m)."""
    gen = SplitMix64(seed)
    vals = _draw_below(gen, m, count * K).reshape(count, K)
    if edges and count:
        pick = gen.take(count) % np.uint64(8)
        for i in range(count):
            k = int(pick[i])
            if k == 0:
                vals[i] = 0
            elif k == 1:
                vals[i] = np.uint64(m - 1)
            elif k == 2:
                vals[i] = 0
                vals[i, K - 1] = np.uint64(m - 1)
    return vals
