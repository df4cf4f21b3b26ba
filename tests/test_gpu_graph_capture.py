"""tft_forward and itft_inverse allocate nothing and can be captured into a graph.

A transform shape the process has not run before is captured straight away
(no eager warm-up of that shape) into one hipGraph: TFT (Alg. 1) of x, a copy
of the transform, then the ITFT (Alg. 2) that undoes it.  The graph is replayed
several times, with eager work (new inputs, other transforms) between the
replays, and every replay is compared with the oracle: the copy must equal
eq. (1) and x must come back as L a_i (Sect. 2: the ITFT leaves the factor L).
"""

import random

import pytest

from oracle import tft_oracle as O
from tests.gpu_util import fermat_from_device, fermat_to_device, fermat_values, nega_from_device, nega_to_device, note

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0810_3203_amd as T  # noqa: E402


def _fermat_case(ring, rng, z):
    p = ring.p
    vals = [rng.randrange(p) for _ in range(z)]
    vals[0] = p - 1       # 2^N
    vals[-1] = (1 << ring.N) - 1
    return vals


# (N, l, s, z, n): two shapes on the first leaf kernel (64 and 256 limbs a
# cell), one on the persistent one (1024 limbs), all of odd truncations not
# used elsewhere
FERMAT_SHAPES = [(2048, 8, 333, 201, 233), (8192, 7, 9001, 101, 117), (32768, 6, 70001, 41, 57)]


@pytest.mark.parametrize("N,l,s,z,n", FERMAT_SHAPES)
def test_fermat_transforms_in_graph(N, l, s, z, n):
    ring = O.FermatRing(N)
    R = T.fermat_ring(N)
    L = 1 << l
    rng = random.Random(N + z)
    wsf = torch.empty(T.transform_workspace(R, 0, l, s, z, n), dtype=torch.uint8, device="cuda")
    wsi = torch.empty(T.transform_workspace(R, 1, l, s, n, n, 0), dtype=torch.uint8, device="cuda")
    a = _fermat_case(ring, rng, z)
    x = fermat_to_device(a + [0] * (L - z), N, L, torch)
    y = torch.empty_like(x)
    note("graph capture fermat N=%d l=%d s=%d z=%d n=%d" % (N, l, s, z, n))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        T.tft_forward(R, l, s, z, n, x, wsf)
        y.copy_(x)
        T.itft_inverse(R, l, s, n, n, 0, x, wsi)
    # capture records the work without running it
    for rep in range(3):
        if rep:
            a = _fermat_case(ring, rng, z)
        x.copy_(fermat_to_device(a + [0] * (L - z), N, L, torch))
        note("replay %d" % rep)
        g.replay()
        torch.cuda.synchronize()
        fwd = fermat_values(*fermat_from_device(y, N, L, n))
        assert fwd == O.tft(ring, L, s, z, n, a), "replay %d: transform differs" % rep
        _, expect = O.itft_case(ring, L, s, n, n, 0, a + [0] * (n - z))
        assert fermat_values(*fermat_from_device(x, N, L, n)) == expect, "replay %d: inverse differs" % rep
        # eager work between replays: another shape through the same entry points
        w = fermat_to_device([1, 2, 3, 4], N, 4, torch)
        T.tft_forward(R, 2, 1, 4, 4, w)
        torch.cuda.synchronize()
        assert fermat_values(*fermat_from_device(w, N, 4, 4)) == O.tft(ring, 4, 1, 4, 4, [1, 2, 3, 4])


def test_nega_transforms_in_graph():
    K, m, l, s, z, n = 64, (1 << 61) - 1, 6, 17, 41, 55
    ring = O.NegaRing(K, m)
    R = T.nega_ring(K, m)
    L = 1 << l
    rng = random.Random(5)
    a = [tuple(rng.randrange(m) for _ in range(K)) for _ in range(z)]
    a[0] = tuple([m - 1] * K)
    wsf = torch.empty(T.transform_workspace(R, 0, l, s, z, n), dtype=torch.uint8, device="cuda")
    wsi = torch.empty(T.transform_workspace(R, 1, l, s, n, n, 0), dtype=torch.uint8, device="cuda")
    x = nega_to_device(a, K, L, torch)
    x0 = x.clone()
    y = torch.empty_like(x)
    note("graph capture nega K=%d l=%d s=%d z=%d n=%d" % (K, l, s, z, n))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        T.tft_forward(R, l, s, z, n, x, wsf)
        y.copy_(x)
        T.itft_inverse(R, l, s, n, n, 0, x, wsi)
    want_fwd = O.tft(ring, L, s, z, n, a)
    _, want_inv = O.itft_case(ring, L, s, n, n, 0, a + [ring.zero()] * (n - z))
    for rep in range(2):
        x.copy_(x0)
        note("replay %d" % rep)
        g.replay()
        torch.cuda.synchronize()
        assert nega_from_device(y, K, n) == want_fwd, "replay %d: transform differs" % rep
        assert nega_from_device(x, K, n) == want_inv, "replay %d: inverse differs" % rep
