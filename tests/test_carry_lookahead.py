"""The carry lookahead used by the bundled unpack: for one round of 64 limb
sums v_l < 2^33 - 1 and a carry c into the round, the carries into the limbs
are the bits of (a + G + c) ^ a ^ G (a = G | P, G the limbs whose sum carries
out, P the limbs whose low word is all ones) and the carry out of the round is
that 64-bit sum's overflow.  Checked against sequential carry propagation on
random and adversarial (long all-ones / carry) patterns."""

import random

M64 = (1 << 64) - 1


def sequential(v, c):
    out, cin = [], []
    for x in v:
        cin.append(c)
        t = x + c
        out.append(t & 0xFFFFFFFF)
        c = t >> 32
        assert c <= 1
    return out, cin, c


def lookahead(v, c):
    G = sum(1 << l for l, x in enumerate(v) if x >> 32)
    P = sum(1 << l for l, x in enumerate(v) if (x & 0xFFFFFFFF) == 0xFFFFFFFF)
    a = G | P
    s = (a + G) & M64
    s2 = (s + c) & M64
    cin = s2 ^ a ^ G
    out = [((x & 0xFFFFFFFF) + ((cin >> l) & 1)) & 0xFFFFFFFF for l, x in enumerate(v)]
    cout = 1 if (s < a or s2 < s) else 0
    return out, [(cin >> l) & 1 for l in range(64)], cout


def _cases():
    rng = random.Random(7)
    full = (1 << 32) - 1
    for _ in range(300):
        yield [rng.randrange(0, 2 * full + 1) for _ in range(64)], rng.randrange(2)
    for _ in range(300):  # runs of all-ones low words fed by carries
        v = []
        for _ in range(64):
            r = rng.random()
            v.append(full if r < 0.6 else (full + 1 + rng.randrange(full) if r < 0.8 else rng.randrange(full)))
        yield v, rng.randrange(2)
    yield [full] * 64, 1  # the carry into the round crosses every limb
    yield [2 * full] + [full] * 63, 0
    yield [0] * 64, 1
    yield [2 * full] * 64, 1


def test_lookahead_matches_sequential_carries():
    for v, c in _cases():
        assert lookahead(v, c) == sequential(v, c)
