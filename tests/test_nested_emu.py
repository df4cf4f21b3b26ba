"""Host run of the nested Schoenhage-Strassen pointwise product.

tests/native/nested_emu.cpp compiles the functions the kernel's nested
pointwise product is made of (paper_0810_3203_amd/csrc/fermat_nested.hpp) for
the host and runs them in the kernel's phase order.  For N = 16384 to 131072
it gets the per-limb positive and negative word sums the kernel's last phase
adds up, and this test checks that they give a b mod 2^N+1 (the oracle's
product in Z/(2^N+1)) for random operands and for the ones that stress the
method: all-ones limbs (the largest pieces and coefficients), a single
nonzero piece at either end, zero, 1, and 2^N - 1.
"""

import os
import random
import subprocess

import pytest

from oracle import tft_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def emu_exe(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("nest") / "nested_emu")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_0810_3203_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", "nested_emu.cpp"), "-o", exe])
    return exe


def _limbs(v, W):
    return [(v >> (32 * q)) & 0xFFFFFFFF for q in range(W)]


def _cases(N, rng):
    W = N // 32
    top = (1 << N) - 1
    piece = 1 << (N // 64)
    vals = [
        (top, top),                                   # every piece and coefficient at its largest
        (rng.getrandbits(N), rng.getrandbits(N)),
        (rng.getrandbits(N), top),
        (0, rng.getrandbits(N)),
        (1, rng.getrandbits(N)),
        (piece - 1, (piece - 1) << (N - N // 64)),    # lowest piece times highest piece
        ((piece - 1) << (N - N // 64), (piece - 1) << (N - N // 64)),
        (rng.getrandbits(N // 2), rng.getrandbits(N)),
        (1 << (N - 1), 1 << (N - 1)),
    ]
    for _ in range(3):
        # runs of ones and zeros at random limb boundaries
        v = 0
        for q in range(W):
            v |= (0xFFFFFFFF if rng.random() < 0.5 else 0) << (32 * q)
        vals.append((v, rng.getrandbits(N)))
    return vals


@pytest.mark.parametrize("N", [16384, 32768, 65536, 131072])
def test_nested_product_emulated(emu_exe, N):
    ring = O.FermatRing(N)
    rng = random.Random(N)
    W = N // 32
    cases = _cases(N, rng)
    inp = ["%d %d" % (W, len(cases))]
    for a, b in cases:
        inp.append(" ".join("%x" % v for v in _limbs(a, W) + _limbs(b, W)))
    r = subprocess.run([emu_exe], input="\n".join(inp) + "\n", capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr
    lines = r.stdout.strip().split("\n")
    assert len(lines) == len(cases)
    p = (1 << N) + 1
    for (a, b), line in zip(cases, lines):
        w = [int(t, 16) for t in line.split()]
        pos, neg = w[:W], w[W:]
        got = sum((pv - nv) << (32 * j) for j, (pv, nv) in enumerate(zip(pos, neg))) % p
        assert got == O.pointwise(ring, [a], [b], 0)[0], (hex(a)[:20], hex(b)[:20])


def test_inner_cell_helpers_emulated(emu_exe):
    """normalize of (L, h) cells with h far outside {0, 1} and at the points
    where the residue wraps to 2^N', and the products involving 2^N' = -1,
    in Z/(2^3072+1) against Python integers."""
    r = subprocess.run([emu_exe], input="0\n", capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    WI = 96
    M = (1 << (32 * WI)) + 1

    def cell(words):
        limbs = [int(t, 16) for t in words[:WI]]
        h = int(words[WI])
        return sum(v << (32 * m) for m, v in enumerate(limbs)), h

    def canonical(v, h):
        return h in (0, 1) and (h == 0 or v == 0) and v < (1 << (32 * WI))

    seen = {"N": 0, "S": 0}
    for line in r.stdout.strip().split("\n"):
        t = line.split()
        kind, t = t[0], t[1:]
        seen[kind] += 1
        if kind == "N":
            L, _ = cell(t[:WI + 1])
            h = int(t[WI + 1])
            v, hv = cell(t[WI + 2:])
            assert canonical(v, hv)
            assert (v + hv * (1 << (32 * WI))) % M == (L - h) % M
        else:
            x, hx = cell(t[:WI + 1])
            y, hy = cell(t[WI + 1:2 * WI + 2])
            v, hv = cell(t[2 * WI + 2:])
            assert canonical(v, hv)
            xv, yv = x + hx * (1 << (32 * WI)), y + hy * (1 << (32 * WI))
            assert (v + hv * (1 << (32 * WI))) % M == xv * yv % M
    assert seen["N"] == 36 and seen["S"] == 12
