"""zx_mul_ss_static (the product run from the library's static device scratch)
gives exactly zx_mul_ss's output, on two calls in a row, the second smaller.

The second call runs over what the first left in the scratch array, so any
dependence on cleared memory shows up as a difference.  Both outputs are also
checked against the schoolbook oracle on sampled coefficients (Sect. 5.1:
the product in Z[x] is exact).
"""

import numpy as np
import pytest

from synth import workloads as wl
from synth.splitmix import SplitMix64
from tests.gpu_util import note, u32_to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0810_3203_amd as T  # noqa: E402


def _out_limbs(lg, gl, lh, hl):
    bits = 32 * (gl + hl) + max(0, (min(lg, lh) - 1).bit_length())
    return (bits + 31) // 32


def _both(g, h, params=None):
    ow = _out_limbs(g.shape[0], g.shape[1], h.shape[0], h.shape[1])
    n = g.shape[0] + h.shape[0] - 1
    gd, hd = u32_to_device(g, torch), u32_to_device(h, torch)
    ref = torch.zeros((n, ow), dtype=torch.int32, device="cuda")
    got = torch.full((n, ow), -1, dtype=torch.int32, device="cuda")
    T.zx_mul_ss(gd, hd, ref, params)
    T.zx_mul_ss_static(gd, hd, got, params)
    torch.cuda.synchronize()
    return ref.cpu().numpy().view(np.uint32), got.cpu().numpy().view(np.uint32), ow


@pytest.mark.parametrize("first,second", [((900, 40, 700, 40), (60, 3, 45, 2)),
                                          ((3000, 63, 3000, 63), (500, 2, 500, 2))])
def test_static_scratch_product_matches_workspace_product(coracle, first, second):
    s = SplitMix64(first[0] + second[0])
    for lg, gl, lh, hl in (first, second):
        g = wl.random_ints(s, lg, 32 * gl)
        h = wl.random_ints(s, lh, 32 * hl)
        g[0] = 0xFFFFFFFF
        h[-1] = 0xFFFFFFFF
        note("zx_mul_ss_static %d x %d limbs, %d x %d limbs" % (lg, gl, lh, hl))
        ref, got, ow = _both(g, h)
        assert np.array_equal(ref, got), "static-scratch product differs from zx_mul_ss"
        ks = sorted({0, 1, lg + lh - 2, (lg + lh) // 2, lg - 1})
        assert np.array_equal(got[ks], coracle.zx_coeffs(g, h, ks, ow))


def test_static_scratch_product_with_explicit_params():
    s = SplitMix64(9)
    g, h = wl.random_ints(s, 611, 300), wl.random_ints(s, 390, 300)
    for p in [T.SSParams(0, 0, T.Split(3, 0), 1, 1), T.SSParams(0, 0, T.Split(0, 2), 2, 0)]:
        note("zx_mul_ss_static params k=%d split %d/%d" % (p.k, p.split.top_l1, p.split.leaf_log2))
        ref, got, _ = _both(g, h, p)
        assert np.array_equal(ref, got)
