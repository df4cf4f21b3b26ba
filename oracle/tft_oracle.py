"""Plain Python oracle (exact integers) — test infrastructure only.

Follows the paper's Sect. 2 ("Notation and setup"):
  * the ring R with a principal root of unity, here
      Z/(2^N+1) with theta = 2 of order 2N       (the Schoenhage-Strassen ring),
      (Z/mZ)[y]/(y^K+1) with theta = y of order 2K (the Schoenhage-Nussbaumer ring,
                                                   Sect. 5.2), or
      Z/pZ, p a word-size prime, with theta of order the largest power of two
      dividing p - 1                            (the small-coefficient case, Sect. 6);
  * omega_L = theta^(ord/L), the principal L-th root (compatibility relation);
  * the weighted DFT, eq. (1), outputs in bit-reversed order;
  * TFT(L, zeta, z, n) = first n outputs of eq. (1) with a_i = 0 for i >= z;
  * ITFT(L, zeta, z, n, f), defined by what it must return;
  * the product in R[X] through TFT, pointwise products and ITFT.
Products in Z[x] and (Z/mZ)[x] are schoolbook.

No blocking, no butterflies, no reordering: every output is the definition
written out.  zeta is passed as an exponent s (zeta = theta^s), the
representation of Sect. 6.
"""

from functools import reduce


def bitrev(j: int, l: int) -> int:
    """Length-l bit reversal of j (the j' of eq. (1))."""
    r = 0
    for _ in range(l):
        r = (r << 1) | (j & 1)
        j >>= 1
    return r


def log2_exact(L: int) -> int:
    l = L.bit_length() - 1
    if L <= 0 or (1 << l) != L:
        raise ValueError("L must be a power of two")
    return l


# ---------------------------------------------------------------------------
# rings (Sect. 2; Sect. 5.1; Sect. 5.2)
# ---------------------------------------------------------------------------

class FermatRing:
    """R = Z/(2^N+1)Z with theta = 2, a principal root of order 2N (Sect. 2, Sect. 5.1).

    Elements are Python ints in canonical form [0, 2^N].
    """

    kind = "fermat"

    def __init__(self, N: int):
        if N < 1:
            raise ValueError("N >= 1")
        self.N = N
        self.p = (1 << N) + 1
        self.ord = 2 * N

    def zero(self):
        return 0

    def canon(self, x):
        return x % self.p

    def add(self, a, b):
        return (a + b) % self.p

    def sub(self, a, b):
        return (a - b) % self.p

    def mul(self, a, b):
        return (a * b) % self.p

    def scal(self, a, k: int):
        """a times the integer k."""
        return (a * k) % self.p

    def theta_pow(self, e: int):
        return pow(2, e % self.ord, self.p)

    def mul_theta(self, a, e: int):
        """a * 2^e, reduced with 2^N = -1: a 2^t = hi 2^N + lo = lo - hi, and 2^(N+t) = -2^t."""
        e %= self.ord
        neg = e >= self.N
        x = (a % self.p) << (e - self.N if neg else e)
        r = ((x & ((1 << self.N) - 1)) - (x >> self.N)) % self.p
        return (-r) % self.p if neg else r

    def inv_pow2(self, k: int):
        """2^-k in R (2 is invertible: 2 * 2^(2N-1) = 2^(2N) = 1)."""
        return pow(2, (-k) % self.ord, self.p)

    def eq(self, a, b):
        return a % self.p == b % self.p


class NegaRing:
    """R = (Z/mZ)[y]/(y^K+1) with theta = y, a principal root of order 2K (Sect. 5.2).

    m is odd, so 2 is invertible.  Elements are tuples of K ints in [0, m),
    coefficient i belonging to y^i.
    """

    kind = "nega"

    def __init__(self, K: int, m: int):
        if K < 1 or m < 3 or m % 2 == 0:
            raise ValueError("K >= 1 and odd m >= 3")
        self.K = K
        self.m = m
        self.ord = 2 * K

    def zero(self):
        return (0,) * self.K

    def canon(self, x):
        return tuple(int(c) % self.m for c in x)

    def add(self, a, b):
        return tuple((x + y) % self.m for x, y in zip(a, b))

    def sub(self, a, b):
        return tuple((x - y) % self.m for x, y in zip(a, b))

    def mul(self, a, b):
        """Negacyclic schoolbook product: y^K = -1."""
        K, m = self.K, self.m
        c = [0] * (2 * K)
        for i, x in enumerate(a):
            if x:
                for j, y in enumerate(b):
                    c[i + j] += x * y
        return tuple((c[k] - c[k + K]) % m for k in range(K))

    def scal(self, a, k: int):
        return tuple((x * k) % self.m for x in a)

    def theta_pow(self, e: int):
        e %= self.ord
        v = [0] * self.K
        if e < self.K:
            v[e] = 1
        else:
            v[e - self.K] = self.m - 1
        return tuple(v)

    def mul_theta(self, a, e: int):
        """a * y^e: coefficient i moves to i + e; passing y^K flips its sign (y^K = -1)."""
        K, m = self.K, self.m
        out = [0] * K
        for i, x in enumerate(a):
            pos = i + (e % self.ord)
            sign = 1
            while pos >= K:
                pos -= K
                sign = -sign
            out[pos] = (sign * x) % m
        return tuple(out)

    def inv_pow2(self, k: int):
        v = [0] * self.K
        v[0] = pow(2, -k, self.m)
        return tuple(v)

    def eq(self, a, b):
        return self.canon(a) == self.canon(b)


class PrimeRing:
    """R = Z/pZ, p an odd prime, with theta = r^((p-1)/2^v): r the smallest
    primitive root mod p and 2^v the largest power of two dividing p - 1, so
    theta has order exactly 2^v (the word-size coefficient ring of Sect. 6).
    Elements are ints in [0, p)."""

    kind = "prime"

    def __init__(self, p: int):
        if p < 3 or p % 2 == 0 or any(p % q == 0 for q in range(3, int(p ** 0.5) + 1, 2)):
            raise ValueError("p must be an odd prime")
        self.p = p
        v = 0
        while (p - 1) % (2 << v) == 0:
            v += 1
        self.ord = 1 << v
        self.r = self._primitive_root()
        self.theta = pow(self.r, (p - 1) >> v, p)

    def _primitive_root(self):
        p = self.p
        n, qs, q = p - 1, [], 2
        while q * q <= n:
            if n % q == 0:
                qs.append(q)
                while n % q == 0:
                    n //= q
            q += 1
        if n > 1:
            qs.append(n)
        for r in range(2, p):
            if all(pow(r, (p - 1) // q, p) != 1 for q in qs):
                return r
        raise ValueError("no primitive root")

    def zero(self):
        return 0

    def canon(self, x):
        return int(x) % self.p

    def add(self, a, b):
        return (a + b) % self.p

    def sub(self, a, b):
        return (a - b) % self.p

    def mul(self, a, b):
        return a * b % self.p

    def scal(self, a, k: int):
        return a * k % self.p

    def theta_pow(self, e: int):
        return pow(self.theta, e % self.ord, self.p)

    def mul_theta(self, a, e: int):
        return a * self.theta_pow(e) % self.p

    def inv_pow2(self, k: int):
        return pow(2, -k, self.p)

    def eq(self, a, b):
        return a % self.p == b % self.p


def omega_exp(ring, L: int) -> int:
    """Exponent e with omega_L = theta^e; needs L | ord(theta) (Sect. 2)."""
    if ring.ord % L:
        raise ValueError("theta has no power of order %d" % L)
    return ring.ord // L


# ---------------------------------------------------------------------------
# transforms (Sect. 2)
# ---------------------------------------------------------------------------

def dft_eq1(ring, L: int, s: int, a, j_list=None):
    """Eq. (1): a_hat_j = zeta^(j') * sum_i omega_L^(i j') a_i, zeta = theta^s.

    ``a`` lists a_0..a_{len(a)-1}; missing a_i (i >= len(a)) are zero.
    Returns the outputs for j in ``j_list`` (default: all j < L).
    """
    l = log2_exact(L)
    w = omega_exp(ring, L)
    if j_list is None:
        j_list = range(L)
    out = []
    for j in j_list:
        jr = bitrev(j, l)
        acc = ring.zero()
        for i, ai in enumerate(a):
            acc = ring.add(acc, ring.mul_theta(ai, w * i * jr))
        out.append(ring.mul_theta(acc, s * jr))
    return out


def tft(ring, L: int, s: int, z: int, n: int, a):
    """TFT(L, zeta, z, n; a_0..a_{z-1}) = (a_hat_0..a_hat_{n-1}), a_i = 0 for i >= z (Sect. 2)."""
    if not (1 <= z <= L and 1 <= n <= L):
        raise ValueError("need 1 <= z, n <= L")
    return dft_eq1(ring, L, s, list(a)[:z], range(n))


def itft_case(ring, L: int, s: int, z: int, n: int, f: int, a):
    """The ITFT of Sect. 2, by its definition.

    Given a_0..a_{z-1} (a_i = 0 for i >= z) returns (inputs, expected):
      inputs   = (a_hat_0..a_hat_{n-1}, L a_n, ..., L a_{z-1})
      expected = (L a_0, ..., L a_{n-1}) followed by a_hat_n when f = 1.
    The ITFT is well defined (Sect. 2), so ``expected`` is the only correct answer.
    """
    if f not in (0, 1) or not (1 <= z <= L and z >= n and 1 <= n + f <= L):
        raise ValueError("need f in {0,1}, 1 <= z <= L, z >= n, 1 <= n+f <= L")
    a = list(a)[:z]
    ahat = dft_eq1(ring, L, s, a, range(n + f))
    inputs = ahat[:n] + [ring.scal(a[i], L) for i in range(n, z)]
    expected = [ring.scal(a[i], L) for i in range(n)] + (ahat[n:n + 1] if f else [])
    return inputs, expected


def pointwise(ring, a, b, scale_log2: int = 0):
    """c_i = a_i b_i 2^(-scale_log2) in R (the n pointwise products of Sect. 2)."""
    t = ring.inv_pow2(scale_log2)
    return [ring.mul(ring.mul(x, y), t) for x, y in zip(a, b)]


def rx_mul_schoolbook(ring, g, h):
    """Schoolbook product in R[X]."""
    n = len(g) + len(h) - 1
    out = [ring.zero() for _ in range(n)]
    for i, x in enumerate(g):
        for j, y in enumerate(h):
            out[i + j] = ring.add(out[i + j], ring.mul(x, y))
    return out


# ---------------------------------------------------------------------------
# polynomial products over the integers and mod m (Sect. 5)
# ---------------------------------------------------------------------------

def zx_mul(g, h):
    """Schoolbook product in Z[x]: u_k = sum_i g_i h_{k-i}."""
    g = [int(x) for x in g]
    h = [int(x) for x in h]
    out = [0] * (len(g) + len(h) - 1)
    for i, x in enumerate(g):
        if x:
            for j, y in enumerate(h):
                out[i + j] += x * y
    return out


def zx_coeff(g, h, k: int) -> int:
    """One coefficient u_k of the Z[x] product, by its sum."""
    lo = max(0, k - (len(h) - 1))
    hi = min(k, len(g) - 1)
    return sum(int(g[i]) * int(h[k - i]) for i in range(lo, hi + 1))


def zmx_mul(g, h, m: int):
    """Schoolbook product in (Z/mZ)[x]."""
    g = [int(x) % m for x in g]
    h = [int(x) % m for x in h]
    out = [0] * (len(g) + len(h) - 1)
    for i, x in enumerate(g):
        if x:
            for j, y in enumerate(h):
                out[i + j] = (out[i + j] + x * y) % m
    return out


def zmx_coeff(g, h, m: int, k: int) -> int:
    lo = max(0, k - (len(h) - 1))
    hi = min(k, len(g) - 1)
    return sum(int(g[i]) * int(h[k - i]) for i in range(lo, hi + 1)) % m


def poly_eval_mod(coeffs, P: int, r: int) -> int:
    """sum_k c_k r^k mod P (Horner).  Used for Schwartz-Zippel fingerprints."""
    return reduce(lambda acc, c: (acc * r + int(c)) % P, reversed(list(coeffs)), 0)
