"""The host planner's expansion of Alg. 1 and Alg. 2, checked on the CPU.

The schedule exported by the library is executed with exact arithmetic
(tests/plan_sim.py) and compared with the oracle's eq. (1) / ITFT definition,
for both rings, many (z, n, f, zeta) and every split policy.  Base-case counts
are checked against Theorems 1 and 2, and the phase structure against the
shapes of Fig. 7 and the partition example of Sect. 6.
"""

import os
import random

import pytest

import paper_0810_3203_amd as T
from oracle import tft_oracle as O
from tests.plan_sim import simulate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand(ring, rng):
    if ring.kind == "fermat":
        # canonical residues including the extreme ones
        k = rng.randrange(8)
        if k == 0:
            return ring.p - 1  # 2^N
        if k == 1:
            return 0
        return rng.randrange(ring.p)
    if ring.kind == "prime":
        return rng.randrange(ring.p)
    return tuple(rng.randrange(ring.m) for _ in range(ring.K))


def _lib_ring(ring):
    if ring.kind == "prime":
        return T.prime_ring()
    return T.fermat_ring(ring.N) if ring.kind == "fermat" else T.nega_ring(ring.K, ring.m)


def _check_tft(ring, l, s, z, n, top_l1=0, leaf_log2=0, seed=0):
    rng = random.Random(seed)
    L = 1 << l
    a = [_rand(ring, rng) for _ in range(L)]  # cells >= z hold garbage
    plan = T.Plan(_lib_ring(ring), 0, l, s, z, n, 0, top_l1, leaf_log2)
    x = simulate(plan.export(), ring, list(a), seed + 1)
    assert x[:n] == O.tft(ring, L, s, z, n, a[:z]), (l, s, z, n, top_l1, leaf_log2)
    return plan


def _check_itft(ring, l, s, z, n, f, top_l1=0, leaf_log2=0, seed=0):
    rng = random.Random(seed)
    L = 1 << l
    a = [_rand(ring, rng) for _ in range(z)]
    inputs, expect = O.itft_case(ring, L, s, z, n, f, a)
    x = list(inputs) + [_rand(ring, rng) for _ in range(L - z)]
    plan = T.Plan(_lib_ring(ring), 1, l, s, z, n, f, top_l1, leaf_log2)
    x = simulate(plan.export(), ring, x, seed + 1)
    assert x[:n + f] == expect, (l, s, z, n, f, top_l1, leaf_log2)
    return plan


FERMAT = O.FermatRing(64)     # ord 128
NEGA = O.NegaRing(16, 1000003)  # ord 32


@pytest.mark.parametrize("leaf_log2", [1, 2, 3, 0])
def test_tft_schedule_matches_eq1_fermat(leaf_log2):
    rng = random.Random(leaf_log2)
    for l in (1, 2, 3, 4, 5, 6):
        L = 1 << l
        cases = {(1, 1), (L, L), (1, L), (L, 1)}
        while len(cases) < min(8, L * L):
            cases.add((rng.randint(1, L), rng.randint(1, L)))
        for z, n in sorted(cases):
            s = rng.randrange(128)
            _check_tft(FERMAT, l, s, z, n, 0, leaf_log2, seed=z * 131 + n)


@pytest.mark.parametrize("leaf_log2", [1, 2, 3, 0])
def test_itft_schedule_matches_definition_fermat(leaf_log2):
    rng = random.Random(100 + leaf_log2)
    for l in (1, 2, 3, 4, 5, 6):
        L = 1 << l
        cases = set()
        for z in {1, L, rng.randint(1, L), rng.randint(1, L)}:
            for n in {0, z, rng.randint(0, z), max(0, z - 1)}:
                for f in (0, 1):
                    if 1 <= n + f <= L:
                        cases.add((z, n, f))
        for z, n, f in sorted(cases):
            s = rng.randrange(128)
            _check_itft(FERMAT, l, s, z, n, f, 0, leaf_log2, seed=z * 7 + n)


@pytest.mark.parametrize("top_l1", [1, 2, 3, 4])
def test_every_top_split_gives_the_same_outputs(top_l1):
    rng = random.Random(top_l1)
    l = 5
    for _ in range(6):
        z, n = rng.randint(1, 32), rng.randint(1, 32)
        _check_tft(FERMAT, l, rng.randrange(128), z, n, top_l1, 2, seed=z + 100 * n)
        zi = rng.randint(1, 32)
        ni = rng.randint(0, zi)
        f = rng.randint(0 if ni else 1, 1 if ni < 32 else 0)
        _check_itft(FERMAT, l, rng.randrange(128), zi, ni, f, top_l1, 2, seed=zi + 100 * ni)


def _column_outputs(ring, l, l1, s, z, a, rows):
    """Eq. (b-cols): output i1 < rows of the column transform of column u, i.e.
    TFT(L1, zeta omega_L^u, z_u, rows) of a_u, a_{u+L2}, ... (a_i = 0 for i >= z)."""
    L, L1, L2 = 1 << l, 1 << l1, 1 << (l - l1)
    z1, z2 = divmod(z, L2)
    b = {}
    for u in range(L2 if z1 else z2):
        col = [a[u + j * L2] for j in range(L1) if u + j * L2 < z]
        for i1, v in enumerate(O.tft(ring, L1, s + (ring.ord // L) * u, len(col), rows, col)):
            b[(i1, u)] = v
    return b


def _first_pass(plan, ring, x, seed):
    d = plan.export()
    return simulate(dict(d, passes=d["passes"][:1]), ring, x, seed), len(d["passes"])


@pytest.mark.parametrize("z,n,s", [(64, 64, 0), (41, 57, 5), (9, 30, 100), (64, 17, 77)])
def test_tft_column_pass_state_is_eq_b_cols(z, n, s):
    """After the top-level column pass of Alg. 1 (L1 = L2 = 8, leaves of 8 cells),
    cell (i1, u) holds eq. (b-cols) for i1 < n1' and u < z2'."""
    ring, l, l1 = FERMAT, 6, 3
    L2 = 1 << (l - l1)
    rng = random.Random(z * 7 + n)
    a = [_rand(ring, rng) for _ in range(1 << l)]
    rows = -(-n // L2)
    x, npass = _first_pass(T.Plan(_lib_ring(ring), 0, l, s, z, n, 0, l1, 3), ring, list(a), 3)
    assert npass == 2
    b = _column_outputs(ring, l, l1, s, z, a, rows)
    for (i1, u), v in b.items():
        assert x[i1 * L2 + u] == v, (i1, u)


@pytest.mark.parametrize("n,s", [(64, 0), (57, 9), (16, 3), (40, 120)])
def test_itft_row_phase_state_is_l2_b(n, s):
    """After the full-row phase of Alg. 2 (z = n, f = 0), full row u < n1 holds
    L2 times the column-pass values b of eq. (b-cols) (the invariant of Sect. 4)."""
    ring, l, l1 = FERMAT, 6, 3
    L2, l2 = 1 << (l - l1), l - l1
    rng = random.Random(n + 1000 * s)
    a = [_rand(ring, rng) for _ in range(n)]
    inputs, _ = O.itft_case(ring, 1 << l, s, n, n, 0, a)
    x = list(inputs) + [_rand(ring, rng) for _ in range((1 << l) - n)]
    x, _ = _first_pass(T.Plan(_lib_ring(ring), 1, l, s, n, n, 0, l1, 3), ring, x, 4)
    n1 = n // L2
    b = _column_outputs(ring, l, l1, s, n, a + [0] * ((1 << l) - n), n1)
    for u in range(n1):
        for i2 in range(L2):
            assert x[u * L2 + i2] == ring.mul_theta(b[(u, i2)], l2), (u, i2)


@pytest.mark.parametrize("leaf_log2", [1, 2, 3])
def test_divide_and_conquer_split_gives_the_same_outputs(leaf_log2):
    """L1 = 2 at every level above the leaf (van der Hoeven's order, Sect. 1)."""
    rng = random.Random(40 + leaf_log2)
    for ring, ordv in ((FERMAT, 128), (NEGA, 32)):
        for l in (2, 4, 5):
            L = 1 << l
            for _ in range(4):
                z, n = rng.randint(1, L), rng.randint(1, L)
                _check_tft(ring, l, rng.randrange(ordv), z, n, T.SPLIT_DC, leaf_log2, seed=z + 31 * n)
                zi = rng.randint(1, L)
                ni = rng.randint(0, zi)
                f = 1 if ni == 0 else (0 if ni == L else rng.randint(0, 1))
                _check_itft(ring, l, rng.randrange(ordv), zi, ni, f, T.SPLIT_DC, leaf_log2, seed=zi + 31 * ni)


def test_divide_and_conquer_matches_the_leaf_recursion():
    """A leaf runs the same L1 = 2 recursion inside LDS, so the divide-and-conquer
    plan with leaves of length 2 performs exactly the base cases of one leaf
    holding the whole transform; its TFT takes l - leaf + 1 passes."""
    rng = random.Random(77)
    ring = T.fermat_ring(2048)  # ord 4096
    for l in range(2, 12):
        L = 1 << l
        for _ in range(4):
            z, n = rng.randint(1, L), rng.randint(1, L)
            dc = T.Plan(ring, 0, l, 0, z, n, 0, T.SPLIT_DC, 1)
            assert dc.base_cases == T.Plan(ring, 0, l, 0, z, n, 0, 0, l).base_cases, (l, z, n)
            zi = rng.randint(1, L)
            ni = rng.randint(0, zi)
            f = 1 if ni == 0 else (0 if ni == L else rng.randint(0, 1))
            dci = T.Plan(ring, 1, l, 0, zi, ni, f, T.SPLIT_DC, 1)
            assert dci.base_cases == T.Plan(ring, 1, l, 0, zi, ni, f, 0, l).base_cases, (l, zi, ni, f)
        for leaf in (1, 3):
            if l > leaf:
                assert len(T.Plan(ring, 0, l, 0, L, L, 0, T.SPLIT_DC, leaf).export()["passes"]) == l - leaf + 1


def test_nega_ring_schedules():
    rng = random.Random(5)
    for l in (1, 3, 5):
        L = 1 << l
        for _ in range(5):
            z, n = rng.randint(1, L), rng.randint(1, L)
            _check_tft(NEGA, l, rng.randrange(32), z, n, 0, rng.choice([1, 2, 0]), seed=z + n)
            zi = rng.randint(1, L)
            ni = rng.randint(0, zi)
            f = 1 if ni == 0 else rng.randint(0, 1 if ni < L else 0)
            _check_itft(NEGA, l, rng.randrange(32), zi, ni, f, 0, rng.choice([1, 2, 0]), seed=zi + ni)


def test_polynomial_product_through_the_schedule():
    """Sect. 2: TFT(g), TFT(h), n products, ITFT(L, 1, n, n, 0) gives L (g h)."""
    ring = FERMAT
    rng = random.Random(8)
    l, L = 6, 64
    g = [rng.randrange(1 << 20) for _ in range(21)]
    h = [rng.randrange(1 << 20) for _ in range(30)]
    n = len(g) + len(h) - 1
    pg = T.Plan(_lib_ring(ring), 0, l, 0, len(g), n, 0, 0, 2).export()
    ph = T.Plan(_lib_ring(ring), 0, l, 0, len(h), n, 0, 0, 2).export()
    xg = simulate(pg, ring, g + [0] * (L - len(g)))
    xh = simulate(ph, ring, h + [0] * (L - len(h)))
    u = [ring.mul(a, b) for a, b in zip(xg[:n], xh[:n])] + [0] * (L - n)
    pi = T.Plan(_lib_ring(ring), 1, l, 0, n, n, 0, 0, 2).export()
    u = simulate(pi, ring, u)
    assert [ring.mul(v, ring.inv_pow2(l)) for v in u[:n]] == O.zx_mul(g, h)


@pytest.mark.parametrize("s", [1, 77, 96, 127])
def test_any_twist_gives_the_same_product(s):
    """Sect. 2 with TFT(g), TFT(h) twisted by zeta = theta^s: by eq. (1) product j
    carries zeta^(2 j'), so the ITFT with zeta^2 still returns L (g h)."""
    ring = FERMAT
    rng = random.Random(s)
    l, L = 6, 64
    g = [rng.randrange(1 << 20) for _ in range(25)]
    h = [rng.randrange(1 << 20) for _ in range(19)]
    n = len(g) + len(h) - 1
    xg = simulate(T.Plan(_lib_ring(ring), 0, l, s, len(g), n, 0, 0, 2).export(), ring, g + [0] * (L - len(g)))
    xh = simulate(T.Plan(_lib_ring(ring), 0, l, s, len(h), n, 0, 0, 2).export(), ring, h + [0] * (L - len(h)))
    assert xg[:n] == O.tft(ring, L, s, len(g), n, g)
    u = [ring.mul(a, b) for a, b in zip(xg[:n], xh[:n])] + [0] * (L - n)
    u = simulate(T.Plan(_lib_ring(ring), 1, l, 2 * s, n, n, 0, 0, 2).export(), ring, u)
    assert [ring.mul(v, ring.inv_pow2(l)) for v in u[:n]] == O.zx_mul(g, h)


@pytest.mark.parametrize("top_l1", [0, 2, T.SPLIT_DC])
def test_whole_row_padding_through_the_schedule(top_l1):
    """Sect. 6 zero-padding: with n rounded up to whole rows of the top split the
    same three transforms give L (g h) followed by zeros, and the ITFT plan has
    no partial last row, so it needs fewer passes."""
    ring = FERMAT
    rng = random.Random(9 + (top_l1 & 7))
    l, L = 6, 64
    l1 = 1 if top_l1 == T.SPLIT_DC else (top_l1 or l // 2)
    L2 = L >> l1
    for lg, lh in ((21, 30), (5, 9), (17, 17)):
        g = [rng.randrange(1 << 20) for _ in range(lg)]
        h = [rng.randrange(1 << 20) for _ in range(lh)]
        n = lg + lh - 1
        npad = -(-n // L2) * L2
        pg = T.Plan(_lib_ring(ring), 0, l, 0, lg, npad, 0, top_l1, 2).export()
        ph = T.Plan(_lib_ring(ring), 0, l, 0, lh, npad, 0, top_l1, 2).export()
        xg = simulate(pg, ring, g + [0] * (L - lg))
        xh = simulate(ph, ring, h + [0] * (L - lh))
        u = [ring.mul(a, b) for a, b in zip(xg[:npad], xh[:npad])] + [rng.randrange(ring.p) for _ in range(L - npad)]
        pi = T.Plan(_lib_ring(ring), 1, l, 0, npad, npad, 0, top_l1, 2)
        u = simulate(pi.export(), ring, u)
        assert [ring.mul(v, ring.inv_pow2(l)) for v in u[:npad]] == O.zx_mul(g, h) + [0] * (npad - n)
        if n % L2:
            plain = T.Plan(_lib_ring(ring), 1, l, 0, n, n, 0, top_l1, 2).export()
            assert len(pi.export()["passes"]) <= len(plain["passes"])


def test_whole_row_padding_pass_counts_large_case():
    """Z/(2^65536+1), L = 2^17, n = 99999: padding to 100352 = 196 rows of 512
    takes the ITFT from 19 passes to 7 with leaves of 16 cells."""
    ring = T.fermat_ring(65536)
    assert len(T.Plan(ring, 1, 17, 0, 99999, 99999, 0, 0, 4).export()["passes"]) == 19
    assert len(T.Plan(ring, 1, 17, 0, 100352, 100352, 0, 0, 4).export()["passes"]) == 7


# ---------------------------------------------------------------------------
# base-case counts (Theorems 1 and 2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("leaf_log2,top", [(1, 0), (0, 0), (1, T.SPLIT_DC), (3, T.SPLIT_DC)])
def test_base_case_counts_within_theorem_bounds(leaf_log2, top):
    rng = random.Random(leaf_log2 + 9 + (top & 1))
    ring = T.fermat_ring(2048)  # ord 4096
    for l in range(1, 13):
        L = 1 << l
        for _ in range(6):
            z, n = rng.randint(1, L), rng.randint(1, L)
            p = T.Plan(ring, 0, l, 0, z, n, 0, top, leaf_log2)
            # Theorem 1: at most min((n-1) l/2 + L - 1, L l/2)
            assert 2 * p.base_cases <= min((n - 1) * l + 2 * (L - 1), L * l), (l, z, n, p.base_cases)
            zi = rng.randint(1, L)
            ni = rng.randint(0, zi)
            f = 1 if ni == 0 else (0 if ni == L else rng.randint(0, 1))
            q = T.Plan(ring, 1, l, 0, zi, ni, f, top, leaf_log2)
            # Theorem 2: at most min((n+f-1) l/2 + L - 1, L l/2)
            assert 2 * q.base_cases <= min((ni + f - 1) * l + 2 * (L - 1), L * l), (l, zi, ni, f, q.base_cases)


# Exact counts with the paper's split at every level (leaf length 2), for the
# benchmark shapes: (ring, l, z, n) -> (TFT count, ITFT count with z = n, f = 0).
EXACT = [
    (T.fermat_ring(512), 10, 500, 999, 5064, 5076),
    (T.fermat_ring(4096), 13, 3000, 5999, 40408, 41504),
    (T.nega_ring(1024, 3), 11, 977, 1953, 10976, 11023),
]


@pytest.mark.parametrize("ring,l,z,n,ct,ci", EXACT)
def test_exact_counts_paper_split(ring, l, z, n, ct, ci):
    assert T.Plan(ring, 0, l, 0, z, n, 0, 0, 1).base_cases == ct
    assert T.Plan(ring, 1, l, 0, n, n, 0, 0, 1).base_cases == ci


def test_exact_counts_large_case():
    ring = T.fermat_ring(65536)
    assert T.Plan(ring, 0, 17, 0, 50000, 99999, 0, 0, 1).base_cases == 893504
    assert T.Plan(ring, 1, 17, 0, 99999, 99999, 0, 0, 1).base_cases == 909040


# ---------------------------------------------------------------------------
# phase structure: Fig. 7 and Sect. 6
# ---------------------------------------------------------------------------

def test_fig7_cases_phase_structure():
    rows = [ln for ln in open(os.path.join(GOLDEN, "itft_fig7_cases.txt")) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 4
    for ln in rows:
        head, tail = ln.split("|")
        _, z, n = head.split()
        expect = [int(v) for v in tail.split()]
        d = T.Plan(T.fermat_ring(1024), 1, 6, 0, int(z), int(n), 0, 0, 3).export()
        assert [p[1] for p in d["passes"]] == expect, ln


def test_sec6_partition():
    ln = [ln for ln in open(os.path.join(GOLDEN, "sec6_partition.txt")) if ln.strip() and not ln.startswith("#")][0]
    head, tail = ln.split("|")
    l, l1, n = (int(v) for v in head.split())
    full, part = (int(v) for v in tail.split())
    d = T.Plan(T.fermat_ring(32 * 256), 0, l, 0, n, n, 0, 0, l1).export()
    assert len(d["passes"]) == 2
    jb, jc, _ = d["passes"][1]
    stores = [j[5] for j in d["jobs"][jb:jb + jc]]
    assert stores.count(1 << (l - l1)) == full and stores.count(part) == 1 and len(stores) == full + 1


PRIME = O.PrimeRing(T.PRIME_P)  # ord 2^27


@pytest.mark.parametrize("leaf_log2", [1, 2, 3])
def test_prime_balanced_schedules(leaf_log2):
    """Z/pZ plans split sub-transforms above the leaf into the fewest passes,
    as evenly as they allow; with small leaves that rule runs several levels
    deep, and the schedules must still give eq. (1) and the ITFT's definition."""
    rng = random.Random(leaf_log2 + 40)
    for l in (5, 7, 9):
        L = 1 << l
        for z, n in {(L, L), (1, L), (rng.randint(1, L), rng.randint(1, L))}:
            _check_tft(PRIME, l, rng.randrange(1 << 27), z, n, 0, leaf_log2, seed=z + n)
        z = rng.randint(2, L)
        n = rng.randint(0, z - 1)
        _check_itft(PRIME, l, rng.randrange(1 << 27), z, n, 1, 0, leaf_log2, seed=z * 3 + n)
        _check_itft(PRIME, l, 5, L, L, 0, 0, leaf_log2, seed=l)


def test_prime_default_plan_shapes():
    """Default Z/pZ plans: leaves of 2^12 words and balanced sub-splits, so a
    transform of 2^24 takes two passes of 4096 jobs of 4096 cells (the paper's
    split at the top), and 2^27 = 13 + 14 levels takes four passes with no job
    below 2^6 cells."""
    ring = T.prime_ring()
    e = T.Plan(ring, 0, 24, 0, 1 << 23, (1 << 24) - 1).export()
    assert e["leaf_log2"] == 12
    assert [(c, m) for _, c, m in e["passes"]] == [(4096, 4096), (4096, 4096)]
    assert {e["progs"][j[2]][2] for j in e["jobs"]} == {4096}
    e = T.Plan(ring, 1, 24, 0, (1 << 24) - 1, (1 << 24) - 1, 0).export()
    assert [c for _, c, _ in e["passes"]] == [4095, 1, 1, 4095]
    e = T.Plan(ring, 0, 27, 0, 1 << 27, 1 << 27).export()
    assert len(e["passes"]) == 4
    assert min(e["progs"][j[2]][2] for j in e["jobs"]) >= 1 << 6
