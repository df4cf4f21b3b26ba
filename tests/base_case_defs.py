"""Operand generators and the definitions of the L = 2 base cases of Alg. 1 and
Alg. 2 in Z/(2^N+1), shared by the emulated and the on-device base-case tests.

The definitions are the base cases as the algorithms state them (Python
integers, no part of the kernels):
  TFT  z=2 n=2: (x0 + x1, zeta (x0 - x1));  z=1 n=2: x1 = zeta x0;  z=2 n=1: x0 + x1
  ITFT n=2: (x0 + x1/zeta, x0 - x1/zeta);  n=1 f=1: (2 x0 - x1, zeta (x0 - x1)),
  with z=1 (2 x0, zeta x0);  n=1 f=0: 2 x0 - x1, or 2 x0;  n=0: (x0 + x1)/2, x0/2.
"""

import random


def expect(code, N, s, x0, x1):
    """(x0', x1') after base case `code` with zeta = 2^s; None where a cell is not an output."""
    p = (1 << N) + 1
    z = pow(2, s, p)
    zi = pow(z, -1, p)
    half = pow(2, -1, p)
    table = {
        1: lambda: ((x0 + x1) % p, z * (x0 - x1) % p),
        2: lambda: (x0, z * x0 % p),
        3: lambda: ((x0 + x1) % p, x1),
        4: lambda: ((x0 + x1 * zi) % p, (x0 - x1 * zi) % p),
        5: lambda: ((2 * x0 - x1) % p, z * (x0 - x1) % p),
        6: lambda: (2 * x0 % p, z * x0 % p),
        7: lambda: ((2 * x0 - x1) % p, None),
        8: lambda: (2 * x0 % p, x1),
        9: lambda: ((x0 + x1) * half % p, x1),
        10: lambda: (x0 * half % p, x1),
    }
    return table[code]()


def operand(rng: random.Random, N: int, kind: int) -> int:
    """Canonical residues of several shapes: random, 0, 1, 2^N, 2^N - 1, one
    half filled, lane chunks of zeros or ones, single limbs, runs of ones."""
    W = N // 32
    C = W // 64
    if kind == 0:
        return rng.randrange((1 << N) + 1)
    if kind == 1:
        return 0
    if kind == 2:
        return 1
    if kind == 3:
        return 1 << N
    if kind == 4:
        return (1 << N) - 1
    if kind == 5:
        return rng.getrandbits(N // 2)
    if kind == 6:
        return rng.getrandbits(N // 2) << (N // 2)
    if kind == 7:
        v = 0
        for ln in range(64):
            if rng.getrandbits(1):
                v |= ((1 << (32 * C)) - 1) << (32 * C * ln)
        return v ^ (rng.getrandbits(32) << (32 * rng.randrange(W)))
    if kind == 8:
        return rng.getrandbits(32) << (32 * rng.randrange(W))
    if kind == 9:
        return (1 << N) - (1 << (32 * rng.randrange(W)))
    return rng.getrandbits(N) >> (32 * rng.randrange(W))


def cases(N: int, count: int, seed: int):
    """(code, s, x0, x1) tuples: every opcode, boundary and random exponents,
    operand kinds paired at random or equal (both operands sparse)."""
    rng = random.Random(seed)
    W = N // 32
    C = W // 64
    special = [0, 1, 31, 32, 33, 32 * C - 1, 32 * C, 32 * C + 1, N - 1, N, N + 1, 2 * N - 1, N // 2, 3 * N // 2, 7,
               7 * 64, 1000]
    out = []
    for i in range(count):
        code = 1 + i % 10
        s = special[(i // 10) % len(special)] if (i // 10) % 2 == 0 else rng.randrange(2 * N)
        k0 = rng.randrange(11)
        k1 = k0 if rng.getrandbits(1) else rng.randrange(11)
        out.append((code, s, operand(rng, N, k0), operand(rng, N, k1)))
    return out
