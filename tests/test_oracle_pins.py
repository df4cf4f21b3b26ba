"""Pins of the CPU oracle against facts other than itself.

Each test ties an oracle function to something the paper or mathematics fixes:
hand-worked values (tests/golden), the principal-root identity of Sect. 2, the
textbook DFT as polynomial evaluation (Sect. 2: z = n = L, zeta = 1), the
paper's closed-form base cases (Alg. 1 and Alg. 2, L = 2), brute-force
uniqueness of the ITFT (Sect. 2), the convolution identity behind the product
of Sect. 2, and library routines (Python big-int multiplication, numpy
convolution) for the schoolbook products.  The last tests plant mistakes in the
oracle and check that a pin catches each of them.
"""

import itertools
import os
import random

import numpy as np
import pytest

from oracle import tft_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_elem(ring, rng):
    if ring.kind in ("fermat", "prime"):
        return rng.randrange(ring.p)
    return tuple(rng.randrange(ring.m) for _ in range(ring.K))


def _theta(ring):
    if ring.kind == "prime":
        return ring.theta
    return 2 if ring.kind == "fermat" else tuple(1 if i == 1 else 0 for i in range(ring.K))


def _one(ring):
    return 1 if ring.kind in ("fermat", "prime") else tuple(1 if i == 0 else 0 for i in range(ring.K))


def _neg_one(ring):
    if ring.kind in ("fermat", "prime"):
        return ring.p - 1
    return tuple(ring.m - 1 if i == 0 else 0 for i in range(ring.K))


RINGS = [O.FermatRing(2), O.FermatRing(4), O.FermatRing(8), O.FermatRing(64), O.FermatRing(96),
         O.NegaRing(4, 15), O.NegaRing(8, (1 << 61) + 11), O.PrimeRing(17), O.PrimeRing(97), O.PrimeRing(257)]
WORD_PRIME = 15 * (1 << 27) + 1


# ---------------------------------------------------------------------------
# hand-worked values
# ---------------------------------------------------------------------------

def test_bitrev_matches_string_reversal():
    for l in range(0, 9):
        for j in range(1 << l):
            s = format(j, "0%db" % l) if l else ""
            assert O.bitrev(j, l) == (int(s[::-1], 2) if l else 0)


def test_golden_dft_z5_L4():
    ring = O.FermatRing(2)  # Z/5
    rows = [ln for ln in open(os.path.join(GOLDEN, "dft_z5_L4.txt")) if not ln.startswith("#") and ln.strip()]
    for ln in rows:
        i, vals = ln.split("|")
        a = [0, 0, 0, 0]
        a[int(i)] = 1
        assert O.dft_eq1(ring, 4, 0, a) == [int(v) for v in vals.split()]


def test_golden_dft_z17_L8_weighted():
    ring = O.FermatRing(4)  # Z/17
    vals = [ln for ln in open(os.path.join(GOLDEN, "dft_z17_L8_e1.txt")) if not ln.startswith("#") and ln.strip()]
    expect = [int(v) for v in vals[0].split()]
    assert O.dft_eq1(ring, 8, 1, [0, 1]) == expect


# ---------------------------------------------------------------------------
# ring facts (Sect. 2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ring", RINGS, ids=lambda r: "%s" % r.kind + str(getattr(r, "N", getattr(r, "K", 0))))
def test_theta_power_by_repeated_multiplication(ring):
    x = _one(ring)
    th = _theta(ring)
    for e in range(ring.ord + 3):
        assert ring.eq(ring.theta_pow(e), x)
        x = ring.mul(x, th)


@pytest.mark.parametrize("ring", RINGS, ids=lambda r: "%s" % r.kind + str(getattr(r, "N", getattr(r, "K", 0))))
def test_principal_root_identity(ring):
    """omega_L^L = 1, omega_L^(L/2) = -1 and sum_i omega_L^(ij) = 0 for 0 < j < L (Sect. 2)."""
    Lmax = ring.ord & -ring.ord  # largest power of two dividing ord(theta)
    for l in range(1, Lmax.bit_length()):
        L = 1 << l
        w = ring.theta_pow(O.omega_exp(ring, L))
        pw = [_one(ring)]
        for _ in range(L):
            pw.append(ring.mul(pw[-1], w))
        assert ring.eq(pw[L], _one(ring))
        assert ring.eq(pw[L // 2], _neg_one(ring))
        for j in range(1, L):
            acc = ring.zero()
            for i in range(L):
                acc = ring.add(acc, pw[(i * j) % L])
            assert ring.eq(acc, ring.zero())


def test_fermat_mul_theta_is_product_with_theta_power():
    rng = random.Random(19)
    for N in (2, 4, 8, 64, 96, 512):
        ring = O.FermatRing(N)
        for _ in range(60):
            a = rng.choice([0, 1, ring.p - 1, rng.randrange(ring.p)])
            e = rng.randrange(-2 * ring.ord, 3 * ring.ord)
            assert ring.mul_theta(a, e) == (a * pow(2, e % ring.ord, ring.p)) % ring.p


def test_nega_mul_theta_is_product_with_theta_power():
    ring = O.NegaRing(8, 1000003)
    rng = random.Random(17)
    for e in range(-3, 2 * ring.K + 3):
        a = tuple(rng.randrange(ring.m) for _ in range(ring.K))
        assert ring.mul_theta(a, e) == ring.mul(a, ring.theta_pow(e))


def test_two_is_invertible():
    for ring in RINGS:
        for k in range(0, 5):
            t = ring.inv_pow2(k)
            x = t
            for _ in range(k):
                x = ring.add(x, x)
            assert ring.eq(x, _one(ring))


# ---------------------------------------------------------------------------
# eq. (1) against polynomial evaluation (textbook DFT, Sect. 2)
# ---------------------------------------------------------------------------

def _horner(ring, a, x):
    acc = ring.zero()
    for c in reversed(a):
        acc = ring.add(ring.mul(acc, x), c)
    return acc


def _pow(ring, x, k):
    r = _one(ring)
    for _ in range(k):
        r = ring.mul(r, x)
    return r


@pytest.mark.parametrize("ring", RINGS[:5] + RINGS[5:], ids=lambda r: "%s" % r.kind + str(getattr(r, "N", getattr(r, "K", 0))))
def test_dft_is_evaluation_at_bitreversed_roots(ring):
    rng = random.Random(7)
    L = min(ring.ord, 16)
    l = L.bit_length() - 1
    w = ring.theta_pow(O.omega_exp(ring, L))
    for s in (0, 1, 3):
        zeta = ring.theta_pow(s)
        a = [_rand_elem(ring, rng) for _ in range(L)]
        got = O.dft_eq1(ring, L, s, a)
        for j in range(L):
            jr = int(format(j, "0%db" % l)[::-1], 2)
            x = _pow(ring, w, jr)
            expect = ring.mul(_pow(ring, zeta, jr), _horner(ring, a, x))
            assert ring.eq(got[j], expect)


def test_tft_is_prefix_of_dft_with_zero_tail():
    ring = O.FermatRing(64)
    rng = random.Random(3)
    L = 32
    for z, n in [(1, 1), (5, 9), (32, 32), (17, 3), (32, 1), (1, 32)]:
        a = [rng.randrange(ring.p) for _ in range(z)]
        full = O.dft_eq1(ring, L, 5, a + [0] * (L - z))
        assert O.tft(ring, L, 5, z, n, a + [rng.randrange(ring.p) for _ in range(L - z)]) == full[:n]


# ---------------------------------------------------------------------------
# closed-form base cases (Alg. 1 and Alg. 2 at L = 2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ring", [O.FermatRing(8), O.FermatRing(64), O.NegaRing(4, 15), O.PrimeRing(97)],
                         ids=["z257", "f64", "nega", "p97"])
def test_tft_base_case_closed_forms(ring):
    rng = random.Random(11)
    for s in range(0, ring.ord, max(1, ring.ord // 8)):
        zeta = ring.theta_pow(s)
        x0, x1 = _rand_elem(ring, rng), _rand_elem(ring, rng)
        assert O.tft(ring, 2, s, 2, 2, [x0, x1]) == [ring.add(x0, x1), ring.mul(zeta, ring.sub(x0, x1))]
        assert O.tft(ring, 2, s, 1, 2, [x0]) == [x0, ring.mul(zeta, x0)]
        assert O.tft(ring, 2, s, 2, 1, [x0, x1]) == [ring.add(x0, x1)]
        assert O.tft(ring, 2, s, 1, 1, [x0]) == [x0]


@pytest.mark.parametrize("ring", [O.FermatRing(8), O.FermatRing(64), O.NegaRing(4, 15), O.PrimeRing(97)],
                         ids=["z257", "f64", "nega", "p97"])
def test_itft_base_case_closed_forms(ring):
    """itft_case's expected output equals Alg. 2's base-case formulas applied to its inputs."""
    rng = random.Random(12)
    two = ring.add(_one(ring), _one(ring))
    half = ring.inv_pow2(1)
    for s in range(0, ring.ord, max(1, ring.ord // 8)):
        zeta = ring.theta_pow(s)
        zinv = ring.theta_pow(-s)
        for z in (1, 2):
            for n in (0, 1, 2):
                for f in (0, 1):
                    if not (z >= n and 1 <= n + f <= 2):
                        continue
                    a = [_rand_elem(ring, rng) for _ in range(z)]
                    x, expect = O.itft_case(ring, 2, s, z, n, f, a)
                    x0 = x[0]
                    x1 = x[1] if z == 2 else None
                    if n == 2:
                        t = ring.mul(zinv, x1)
                        got = [ring.add(x0, t), ring.sub(x0, t)]
                    elif n == 1 and z == 2:
                        got = [ring.sub(ring.mul(two, x0), x1)] + ([ring.mul(zeta, ring.sub(x0, x1))] if f else [])
                    elif n == 1 and z == 1:
                        got = [ring.mul(two, x0)] + ([ring.mul(zeta, x0)] if f else [])
                    elif z == 2:
                        got = [ring.mul(half, ring.add(x0, x1))]
                    else:
                        got = [ring.mul(half, x0)]
                    assert got == expect, (s, z, n, f)


# ---------------------------------------------------------------------------
# ITFT is well defined (Sect. 2): brute force in Z/5
# ---------------------------------------------------------------------------

def test_itft_unique_bruteforce_z5():
    ring = O.FermatRing(2)  # Z/5, theta = 2 of order 4
    for L in (2, 4):
        for s in range(4):
            for z in range(1, L + 1):
                for n in range(0, z + 1):
                    for f in (0, 1):
                        if not (1 <= n + f <= L):
                            continue
                        seen = {}
                        for a in itertools.product(range(5), repeat=z):
                            x, _ = O.itft_case(ring, L, s, z, n, f, list(a))
                            key = tuple(x)
                            assert key not in seen, (L, s, z, n, f, a, seen.get(key))
                            seen[key] = a
                        assert len(seen) == 5 ** z


# ---------------------------------------------------------------------------
# the product in R[X] (Sect. 2) and schoolbook products
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ring", [O.FermatRing(64), O.NegaRing(8, 1000003), O.PrimeRing(WORD_PRIME)],
                         ids=["f64", "nega", "wordprime"])
def test_convolution_identity(ring):
    """TFT of the schoolbook product = pointwise product of the TFTs (first n values)."""
    rng = random.Random(5)
    L = 16
    for lg, lh in [(1, 1), (3, 5), (8, 9), (16, 1)]:
        g = [_rand_elem(ring, rng) for _ in range(lg)]
        h = [_rand_elem(ring, rng) for _ in range(lh)]
        u = O.rx_mul_schoolbook(ring, g, h)
        n = len(u)
        lhs = O.tft(ring, L, 0, n, n, u)
        rhs = O.pointwise(ring, O.tft(ring, L, 0, lg, n, g), O.tft(ring, L, 0, lh, n, h))
        assert lhs == rhs


def test_word_prime_ring_facts():
    """p = 15 2^27 + 1 is prime, 31 is its smallest primitive root, theta = 31^15
    has order exactly 2^27 (Sect. 6: roots of unity of every power-of-two order
    up to 2^27 exist in Z/pZ)."""
    p = WORD_PRIME
    assert all(p % q for q in range(2, 44900))  # 44900^2 > p
    ring = O.PrimeRing(p)
    assert ring.ord == 1 << 27 and ring.r == 31
    assert all(pow(31, (p - 1) // q, p) != 1 for q in (2, 3, 5)) and all(pow(r, (p - 1) // 2, p) == 1 or
                                                                        pow(r, (p - 1) // 3, p) == 1 or
                                                                        pow(r, (p - 1) // 5, p) == 1
                                                                        for r in range(2, 31))
    assert ring.theta == pow(31, 15, p)
    assert pow(ring.theta, 1 << 26, p) == p - 1 and pow(ring.theta, 1 << 27, p) == 1
    assert ring.inv_pow2(1) * 2 % p == 1


def test_word_prime_schoolbook_against_numpy_convolve():
    rng = random.Random(21)
    ring = O.PrimeRing(WORD_PRIME)
    for lg, lh in [(1, 1), (7, 3), (40, 33)]:
        g = [rng.randrange(ring.p) for _ in range(lg)]
        h = [rng.randrange(ring.p) for _ in range(lh)]
        want = [int(v) % ring.p for v in np.convolve(np.array(g, dtype=object), np.array(h, dtype=object))]
        assert O.rx_mul_schoolbook(ring, g, h) == want


def test_zx_mul_against_python_bigint_kronecker():
    rng = random.Random(9)
    for lg, lh, bits in [(1, 1, 64), (7, 3, 200), (40, 50, 130)]:
        g = [rng.getrandbits(bits) for _ in range(lg)]
        h = [rng.getrandbits(bits) for _ in range(lh)]
        B = 2 * bits + 16
        G = sum(c << (B * i) for i, c in enumerate(g))
        H = sum(c << (B * i) for i, c in enumerate(h))
        P = G * H
        mask = (1 << B) - 1
        expect = [(P >> (B * k)) & mask for k in range(lg + lh - 1)]
        assert O.zx_mul(g, h) == expect
        for k in (0, lg + lh - 2, (lg + lh - 2) // 2):
            assert O.zx_coeff(g, h, k) == expect[k]


def test_zmx_mul_against_numpy_convolve():
    rng = random.Random(10)
    m = (1 << 61) + 15
    for lg, lh in [(1, 1), (9, 4), (60, 33)]:
        g = [rng.randrange(m) for _ in range(lg)]
        h = [rng.randrange(m) for _ in range(lh)]
        conv = np.convolve(np.array(g, dtype=object), np.array(h, dtype=object))
        expect = [int(c) % m for c in conv]
        assert O.zmx_mul(g, h, m) == expect
        assert O.zmx_coeff(g, h, m, lg - 1) == expect[lg - 1]


def test_nega_mul_against_numpy_convolve_fold():
    rng = random.Random(13)
    K, m = 8, 1000003
    ring = O.NegaRing(K, m)
    for _ in range(20):
        a = tuple(rng.randrange(m) for _ in range(K))
        b = tuple(rng.randrange(m) for _ in range(K))
        c = np.convolve(np.array(a, dtype=object), np.array(b, dtype=object))
        c = list(c) + [0]
        expect = tuple((int(c[k]) - int(c[k + K])) % m for k in range(K))
        assert ring.mul(a, b) == expect


def test_fingerprint_horner():
    P = (1 << 61) - 1
    rng = random.Random(4)
    c = [rng.getrandbits(200) for _ in range(30)]
    r = rng.randrange(P)
    assert O.poly_eval_mod(c, P, r) == sum(x * pow(r, k, P) for k, x in enumerate(c)) % P


# ---------------------------------------------------------------------------
# C oracle against the Python oracle and Python integers
# ---------------------------------------------------------------------------

def _cells_to_ints(limbs, tops):
    N = 32 * limbs.shape[1]
    return [int.from_bytes(limbs[i].tobytes(), "little") + (int(tops[i]) << N) for i in range(limbs.shape[0])]


def test_c_fermat_mul2exp(coracle):
    from synth.workloads import fermat_cells
    for N in (32, 64, 96, 512):
        ring = O.FermatRing(N)
        limbs, tops = fermat_cells(100 + N, 40, N // 32)
        xs = _cells_to_ints(limbs, tops)
        rng = random.Random(N)
        for i, x in enumerate(xs):
            for e in (0, 1, 31, 32, N - 1, N, N + 1, 2 * N - 1, rng.randrange(2 * N)):
                out, top = coracle.fermat_mul2exp(N, limbs[i], tops[i], e)
                got = int.from_bytes(out.tobytes(), "little") + (top << N)
                assert got == ring.mul_theta(x, e), (N, x, e)


def test_c_fermat_dft_matches_python(coracle):
    from synth.workloads import fermat_cells
    for N, L, z, s in [(32, 64, 64, 0), (32, 16, 9, 5), (64, 128, 100, 77), (512, 256, 200, 3)]:
        ring = O.FermatRing(N)
        limbs, tops = fermat_cells(7 * N + L, z, N // 32)
        a = _cells_to_ints(limbs, tops)
        js = list(range(0, L, max(1, L // 24))) + [L - 1]
        ol, ot = coracle.fermat_dft_sampled(N, L, s, limbs, tops, js)
        got = _cells_to_ints(ol, ot)
        assert got == O.dft_eq1(ring, L, s, a, js)


def test_c_nega_dft_matches_python(coracle):
    K, m = 8, (1 << 61) + 11
    ring = O.NegaRing(K, m)
    rng = random.Random(2)
    for L, z, s in [(16, 16, 0), (8, 5, 3), (16, 11, 15)]:
        a = np.array([[rng.randrange(m) for _ in range(K)] for _ in range(z)], dtype=np.uint64)
        js = list(range(L))
        out = coracle.nega_dft_sampled(K, m, L, s, a, js)
        expect = O.dft_eq1(ring, L, s, [tuple(int(v) for v in row) for row in a], js)
        assert [tuple(int(v) for v in row) for row in out] == expect


def test_c_zx_coeffs_match_python(coracle):
    from synth.workloads import random_ints, limbs_to_ints
    from synth.splitmix import SplitMix64
    gen = SplitMix64(99)
    g = random_ints(gen, 23, 100)
    h = random_ints(gen, 17, 70)
    expect = O.zx_mul(limbs_to_ints(g), limbs_to_ints(h))
    ks = list(range(len(expect)))
    got = limbs_to_ints(coracle.zx_coeffs(g, h, ks, 8))
    assert got == expect


def test_c_zmx_and_fingerprint_match_python(coracle):
    rng = random.Random(21)
    m = (1 << 61) + 15
    g = np.array([rng.randrange(m) for _ in range(50)], dtype=np.uint64)
    h = np.array([rng.randrange(m) for _ in range(41)], dtype=np.uint64)
    expect = O.zmx_mul([int(x) for x in g], [int(x) for x in h], m)
    got = coracle.zmx_coeffs(g, h, m, list(range(len(expect))))
    assert [int(x) for x in got] == expect
    P = (1 << 61) - 1
    assert coracle.fingerprint64(np.array(expect, dtype=np.uint64), P, 12345) == O.poly_eval_mod(expect, P, 12345)
    from synth.workloads import ints_to_limbs
    big = [rng.getrandbits(150) for _ in range(12)]
    assert coracle.fingerprint(ints_to_limbs(big, 5), P, 777) == O.poly_eval_mod(big, P, 777)


# ---------------------------------------------------------------------------
# planted mistakes: each must be caught by a pin above
# ---------------------------------------------------------------------------

def _pins_pass():
    try:
        test_golden_dft_z5_L4()
        test_golden_dft_z17_L8_weighted()
        for ring in RINGS[:3]:
            test_principal_root_identity(ring)
            test_dft_is_evaluation_at_bitreversed_roots(ring)
        test_itft_base_case_closed_forms(O.FermatRing(8))
        test_convolution_identity(O.FermatRing(64))
    except AssertionError:
        return False
    return True


def test_c_prime_dft_matches_python(coracle):
    ring = O.PrimeRing(WORD_PRIME)
    rng = random.Random(23)
    for L, s, z in [(2, 0, 2), (16, 3, 11), (256, 12345, 200)]:
        a = [rng.randrange(ring.p) for _ in range(z)]
        js = list(range(L)) if L <= 16 else [0, 1, 7, 100, 255]
        got = [int(v) for v in coracle.prime_dft_sampled(ring, L, s, np.array(a, dtype=np.uint32), js)]
        assert got == O.dft_eq1(ring, L, s, a, js)


def test_pins_pass_unmutated():
    assert _pins_pass()


@pytest.mark.parametrize("mutation", ["bitrev_identity", "omega_off_by_one", "zeta_not_bitreversed",
                                      "itft_drops_scale", "itft_next_coeff_shift", "wrong_modulus_sign"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    if mutation == "bitrev_identity":
        monkeypatch.setattr(O, "bitrev", lambda j, l: j)
    elif mutation == "omega_off_by_one":
        monkeypatch.setattr(O, "omega_exp", lambda ring, L: ring.ord // L + 1)
    elif mutation == "zeta_not_bitreversed":
        orig = O.dft_eq1

        def bad(ring, L, s, a, j_list=None):
            l = O.log2_exact(L)
            w = O.omega_exp(ring, L)
            out = []
            for j in (range(L) if j_list is None else j_list):
                jr = O.bitrev(j, l)
                acc = ring.zero()
                for i, ai in enumerate(a):
                    acc = ring.add(acc, ring.mul_theta(ai, w * i * jr))
                out.append(ring.mul_theta(acc, s * j))
            return out
        monkeypatch.setattr(O, "dft_eq1", bad)
        del orig
    elif mutation == "itft_drops_scale":
        orig = O.itft_case

        def bad(ring, L, s, z, n, f, a):
            x, e = orig(ring, L, s, z, n, f, a)
            half = ring.inv_pow2(1)
            return x, [ring.mul(v, half) if i < n else v for i, v in enumerate(e)]
        monkeypatch.setattr(O, "itft_case", bad)
    elif mutation == "itft_next_coeff_shift":
        orig = O.itft_case

        def bad(ring, L, s, z, n, f, a):
            x, e = orig(ring, L, s, z, n, f, a)
            if f:
                e = e[:n] + [O.dft_eq1(ring, L, s, list(a)[:z], [max(0, n - 1)])[0]]
            return x, e
        monkeypatch.setattr(O, "itft_case", bad)
    elif mutation == "wrong_modulus_sign":
        monkeypatch.setattr(O.FermatRing, "__init__",
                            lambda self, N: (setattr(self, "N", N), setattr(self, "p", (1 << N) - 1),
                                             setattr(self, "ord", 2 * N), None)[-1])
    assert not _pins_pass()
