"""SplitMix64 draws computed by torch on any device (same values as
synth.splitmix), so that large workloads can be generated where they are used.

torch has no full unsigned 64-bit arithmetic, so the state is kept in int64
with two's-complement wrap-around (addition and multiplication mod 2^64 are the
same bits signed or unsigned) and the logical right shifts mask off the sign
copies an arithmetic shift brings in.  Nothing here holds any arithmetic of the
transform or the products.
"""

from .splitmix import GAMMA, _M1, _M2
from .workloads import case_seed


def _s64(v: int) -> int:
    v &= (1 << 64) - 1
    return v - (1 << 64) if v >> 63 else v


def _lsr(torch, z, s):
    return (z >> s) & ((1 << (64 - s)) - 1)


def draws(torch, seed: int, start: int, count: int, device):
    """Draws start+1 .. start+count of the stream `seed` as an int64 tensor (bits of the uint64 values)."""
    idx = torch.arange(start + 1, start + 1 + count, dtype=torch.int64, device=device)
    z = idx * _s64(GAMMA) + _s64(seed)
    z = z ^ _lsr(torch, z, 30)
    z = z * _s64(_M1)
    z = z ^ _lsr(torch, z, 27)
    z = z * _s64(_M2)
    return z ^ _lsr(torch, z, 31)


def ints(torch, seed: int, start: int, count: int, bits: int, device):
    """`count` values of `bits` bits from draws start+1.. (ceil(bits/64) draws each, masked), as an
    int32 tensor (count, ceil(bits/32)) of little-endian limbs; the same values as
    synth.workloads.random_ints on a stream positioned at `start`."""
    d = (bits + 63) // 64
    w = (bits + 31) // 32
    z = draws(torch, seed, start, count * d, device).reshape(count, d)
    limbs = z.view(torch.int32).reshape(count, 2 * d)[:, :w].contiguous()
    rem = bits - 32 * (w - 1)
    if rem < 32:
        limbs[:, w - 1] &= (1 << rem) - 1
    return limbs


def batch_request(torch, i: int, device, bits: int = 1000, len_lo: int = 100, len_hi: int = 20000):
    """Request i of the batch workload (see synth.workloads.batch_request) generated on `device`."""
    seed = case_seed(5) + ((i + 1) << 40)
    lens = draws(torch, seed, 0, 2, "cpu").tolist()
    span = len_hi - len_lo + 1
    lg = len_lo + (lens[0] % (1 << 64)) % span
    lh = len_lo + (lens[1] % (1 << 64)) % span
    d = (bits + 63) // 64
    g = ints(torch, seed, 2, lg, bits, device)
    h = ints(torch, seed, 2 + lg * d, lh, bits, device)
    return g, h
