"""GPU parity of bundled and batched Schoenhage-Strassen products.

- zx_mul_ss with k > 1 coefficients per ring element, against the schoolbook oracle;
- tft_batch_plan_execute (direct launches and hipGraph replays) against the
  oracle and, bit for bit, against one-at-a-time zx_mul_ss with the same
  parameters; per-request status; chunking by workspace limit;
- a sample of the 4096-request workload (lengths uniform in [100, 20000],
  1000-bit coefficients) with the default rule, checked on sampled
  coefficients and Schwartz-Zippel fingerprints.
"""

import random

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

PRIMES = [(1 << 61) - 1, (1 << 62) - 57]


def _out_limbs(lg, gl, lh, hl):
    bits = 32 * (gl + hl) + (min(lg, lh) - 1).bit_length()
    return (bits + 31) // 32


def _operands(seed, lg, lh, bits):
    s = SplitMix64(seed)
    g, h = wl.random_ints(s, lg, bits), wl.random_ints(s, lh, bits)
    g[0] = (1 << 32) - 1
    h[-1] = (1 << 32) - 1
    return g, h


class _Req:
    """Host operands, device tensors and a ZXRequest for one product."""

    def __init__(self, g, h, params=None, out_limbs=None, sentinel=0):
        self.g, self.h = g, h
        self.ow = out_limbs or _out_limbs(g.shape[0], g.shape[1], h.shape[0], h.shape[1])
        self.dg, self.dh = u32_to_device(g, torch), u32_to_device(h, torch)
        self.out = torch.full((g.shape[0] + h.shape[0] - 1, self.ow), sentinel, dtype=torch.int32, device="cuda")
        self.params = params
        self.req = T.zx_request(self.dg, self.dh, self.out, params)

    def result(self):
        return self.out.cpu().numpy().view(np.uint32).copy()

    def one_at_a_time(self):
        o = torch.zeros_like(self.out)
        T.zx_mul_ss(self.dg, self.dh, o, self.params)
        torch.cuda.synchronize()
        return o.cpu().numpy().view(np.uint32)


def _oracle_full(coracle, r):
    return coracle.zx_coeffs(r.g, r.h, range(r.g.shape[0] + r.h.shape[0] - 1), r.ow)


def _fingerprint_ok(coracle, g, h, got, seed):
    rng = random.Random(seed)
    for P in PRIMES:
        x = rng.randrange(2, P - 1)
        if coracle.fingerprint(got, P, x) != coracle.fingerprint(g, P, x) * coracle.fingerprint(h, P, x) % P:
            return False
    return True


@pytest.mark.parametrize("k", [2, 3, 4, 8, 16, 32])
def test_bundled_k_full(coracle, k):
    for lg, lh, bits in [(1, 1, 64), (5, 5, 32), (37, 100, 96), (300, 257, 64), (64, 64, 1000)]:
        g, h = _operands(k * 7919 + lg, lg, lh, bits)
        r = _Req(g, h, T.SSParams(0, 0, T.Split(0, 0), k))
        note("zx_mul_ss k=%d %dx%d %d bits" % (k, lg, lh, bits))
        got = r.one_at_a_time()
        assert np.array_equal(got, _oracle_full(coracle, r)), "k=%d %dx%d" % (k, lg, lh)


@pytest.mark.parametrize("k,bits", [(2, 1000), (3, 1000), (8, 2016), (4, 4000)])
def test_bundled_carry_runs(coracle, k, bits):
    """All-ones coefficients: the slot sums of the bundled unpack carry through
    long runs of all-ones limbs, across rounds of 64 output limbs."""
    for lg, lh in [(7, 9), (40, 33)]:
        w = (bits + 31) // 32
        g = np.full((lg, w), 0xFFFFFFFF, dtype=np.uint32)
        h = np.full((lh, w), 0xFFFFFFFF, dtype=np.uint32)
        top = bits - 32 * (w - 1)
        if top < 32:
            g[:, -1] = (1 << top) - 1
            h[:, -1] = (1 << top) - 1
        h[1::3] = 0  # zero coefficients between the full ones
        r = _Req(g, h, T.SSParams(0, 0, T.Split(0, 0), k))
        note("zx_mul_ss all-ones k=%d %dx%d %d bits (%d output limbs)" % (k, lg, lh, bits, r.ow))
        assert np.array_equal(r.one_at_a_time(), _oracle_full(coracle, r)), "k=%d %dx%d" % (k, lg, lh)


def test_bundled_k_with_split_and_ring(coracle):
    g, h = _operands(99, 200, 150, 64)
    for p in [T.SSParams(0, 0, T.Split(2, 0), 2), T.SSParams(0, 0, T.Split(1, 2), 4),
              T.SSParams(4096, 0, T.Split(0, 0), 4), T.SSParams(0, 9, T.Split(0, 3), 2)]:
        note("zx_mul_ss k=%d N=%d l=%d split %d/%d" % (p.k, p.N, p.l, p.split.top_l1, p.split.leaf_log2))
        r = _Req(g, h, p)
        assert np.array_equal(r.one_at_a_time(), _oracle_full(coracle, r))


def _mixed_requests(seed=2024):
    rng = random.Random(seed)
    reqs = []
    choices = [None, T.SSParams(0, 0, T.Split(0, 0), 1), T.SSParams(0, 0, T.Split(0, 0), 2),
               T.SSParams(0, 0, T.Split(0, 0), 4), T.SSParams(0, 0, T.Split(0, 0), 8),
               T.SSParams(0, 0, T.Split(2, 0), 2), T.SSParams(0, 0, T.Split(0, 3), 1),
               T.SSParams(0, 0, T.Split(0, 0), 1, 1), T.SSParams(0, 0, T.Split(T.SPLIT_DC, 0), 2, 1),
               T.SSParams(0, 0, T.Split(0, 0), 2, 1, 3 << 20)]
    for i in range(21):
        bits = rng.choice([32, 64, 96, 1000])
        hi = 150 if bits == 1000 else 600
        lg, lh = rng.randint(1, hi), rng.randint(1, hi)
        g, h = _operands(seed * 1000 + i, lg, lh, bits)
        p = choices[i % len(choices)]
        if p is not None and p.split.top_l1:
            # keep the explicit split valid for this shape
            p = T.SSParams(0, 0, T.Split(0, 0), p.k) if lg + lh < 16 else p
        reqs.append(_Req(g, h, p))
    return reqs


def test_batch_matches_oracle_and_single(coracle):
    reqs = _mixed_requests()
    plan = T.BatchPlan([r.req for r in reqs])
    assert plan.status() == [0] * len(reqs)
    ws = torch.empty(max(1, plan.workspace), dtype=torch.uint8, device="cuda")
    note("batch plan: %d requests, %d launches, %d bytes" % (len(reqs), plan.launches, plan.workspace))
    plan.execute(ws)
    torch.cuda.synchronize()
    for i, r in enumerate(reqs):
        got = r.result()
        assert np.array_equal(got, _oracle_full(coracle, r)), "request %d vs oracle" % i
        assert np.array_equal(got, r.one_at_a_time()), "request %d vs one-at-a-time" % i


def test_batch_nested_pointwise_sizes(coracle):
    """Batch plans whose rings take the nested pointwise level through the
    item-list kernel at every size it serves: 1000-bit coefficients bundled
    k = 4, 8, 16, 32 per element give 512-, 1024-, 2048- and 4096-limb cells;
    plus one all-ones request.  Against the oracle and one-at-a-time."""
    reqs = []
    for i, k in enumerate((4, 8, 16, 32, 16)):
        lg, lh = 37 + 13 * i, 29 + 7 * i
        g, h = _operands(777 + i, lg, lh, 1000)
        if i == 4:
            g[:] = 0xFFFFFFFF
            h[:] = 0xFFFFFFFF
            g[:, -1] = h[:, -1] = (1 << (1000 - 32 * 31)) - 1
        reqs.append(_Req(g, h, T.SSParams(0, 0, T.Split(0, 0), k)))
    plan = T.BatchPlan([r.req for r in reqs])
    assert plan.status() == [0] * len(reqs)
    ws = torch.empty(max(1, plan.workspace), dtype=torch.uint8, device="cuda")
    note("batch plan of nested pointwise sizes: %d launches" % plan.launches)
    plan.execute(ws)
    torch.cuda.synchronize()
    for i, r in enumerate(reqs):
        got = r.result()
        assert np.array_equal(got, _oracle_full(coracle, r)), "request %d vs oracle" % i
        assert np.array_equal(got, r.one_at_a_time()), "request %d vs one-at-a-time" % i


def test_batch_launch_classes(coracle):
    """Requests of one ring whose passes fall in different work-group classes
    (leaves of 4, 8 and 16 cells, each class with 512 jobs or more a pass, plus
    the batch's own leaf and a short request whose small class joins a larger
    one): pass p then runs in several launches.  Bit for bit against
    one-at-a-time, on oracle samples, and through a graph replay."""
    reqs = []
    for i, leaf in enumerate((2, 3, 4, 0, 2)):
        lg, lh = (4000, 4100) if i < 4 else (60, 45)
        g, h = _operands(4242 + i, lg, lh, 64)
        reqs.append(_Req(g, h, T.SSParams(0, 0, T.Split(0, leaf), 1)))
    plan = T.BatchPlan([r.req for r in reqs])
    assert plan.status() == [0] * len(reqs)
    # the same requests with one leaf size: fewer launches
    same = [_Req(r.g, r.h, T.SSParams(0, 0, T.Split(0, 0), 1)) for r in reqs]
    plan1 = T.BatchPlan([r.req for r in same])
    note("batch launch classes: %d launches (one leaf size: %d)" % (plan.launches, plan1.launches))
    assert plan.launches > plan1.launches
    ws = torch.empty(max(1, plan.workspace), dtype=torch.uint8, device="cuda")
    plan.execute(ws)
    torch.cuda.synchronize()
    rng = random.Random(9)
    for i, r in enumerate(reqs):
        got = r.result()
        assert np.array_equal(got, r.one_at_a_time()), "request %d vs one-at-a-time" % i
        nout = r.g.shape[0] + r.h.shape[0] - 1
        idx = sorted(set([0, nout - 1] + [rng.randrange(nout) for _ in range(24)]))
        exp = coracle.zx_coeffs(r.g, r.h, idx, r.ow)
        assert np.array_equal(got[idx], exp), "request %d vs oracle samples" % i
    ref = [r.result() for r in reqs]
    for r in reqs:
        r.out.zero_()
    note("batch launch classes: graph replay")
    plan.execute(ws, use_graph=True)
    torch.cuda.synchronize()
    for i, r in enumerate(reqs):
        assert np.array_equal(r.result(), ref[i]), "graph replay request %d" % i


def test_batch_graph_replays():
    reqs = _mixed_requests(seed=7)
    plan = T.BatchPlan([r.req for r in reqs])
    ws = torch.empty(plan.workspace, dtype=torch.uint8, device="cuda")
    note("batch eager reference")
    plan.execute(ws)
    torch.cuda.synchronize()
    ref = [r.result() for r in reqs]
    for rep in range(4):
        for r in reqs:
            r.out.zero_()
        noise = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work between replays
        note("batch graph execution %d" % rep)
        plan.execute(ws, use_graph=True)
        torch.cuda.synchronize()
        assert float(noise) == float(noise)
        for i, r in enumerate(reqs):
            assert np.array_equal(r.result(), ref[i]), "replay %d request %d" % (rep, i)


def test_batch_status_and_chunks(coracle):
    g, h = _operands(5, 40, 30, 64)
    good = [_Req(g, h), _Req(h, g, T.SSParams(0, 0, T.Split(0, 0), 4))]
    short = _Req(g, h, out_limbs=2, sentinel=7)                      # output too narrow
    badsplit = _Req(g, h, T.SSParams(0, 0, T.Split(9, 0), 1), sentinel=7)  # top split >= l
    more = [_Req(*_operands(50 + i, 100 + 37 * i, 80, 96)) for i in range(4)]
    allr = good[:1] + [short] + good[1:] + [badsplit] + more
    biggest = max(T.zx_mul_ss_workspace(r.g.shape[0], r.g.shape[1], r.h.shape[0], r.h.shape[1], r.params)
                  for r in good + more)
    biggest = (biggest + 255) // 256 * 256
    plan = T.BatchPlan([r.req for r in allr], max_workspace=biggest)
    st = plan.status()
    assert st[1] == 3 and st[3] == 1 and all(st[i] == 0 for i in (0, 2, 4, 5, 6, 7))
    assert plan.workspace <= biggest
    ws = torch.empty(plan.workspace, dtype=torch.uint8, device="cuda")
    note("batch with skipped requests, chunked at %d bytes" % biggest)
    plan.execute(ws)
    torch.cuda.synchronize()
    for r in (short, badsplit):
        assert (r.result() == 7).all(), "a skipped request's output was written"
    for i, r in enumerate(good + more):
        assert np.array_equal(r.result(), _oracle_full(coracle, r)), "request %d" % i
    with pytest.raises(T.TFTError):
        plan.execute(ws[: plan.workspace - 1])


def test_batch_case5_sample(coracle):
    count = 48
    reqs = []
    for i in range(count):
        g, h = wl.batch_request(i)
        p = T.ss_default_params(g.shape[0], g.shape[1], h.shape[0], h.shape[1])
        reqs.append(_Req(g, h, p))
    plan = T.BatchPlan([r.req for r in reqs])
    ws = torch.empty(plan.workspace, dtype=torch.uint8, device="cuda")
    note("case-5 sample: %d requests, %d launches, %.1f MB workspace" % (count, plan.launches, plan.workspace / 1e6))
    plan.execute(ws, use_graph=True)
    torch.cuda.synchronize()
    rng = random.Random(55)
    for i, r in enumerate(reqs):
        got = r.result()
        n = got.shape[0]
        assert _fingerprint_ok(coracle, r.g, r.h, got, 1000 + i), "request %d fingerprint" % i
        ks = sorted({0, n - 1, rng.randrange(n), rng.randrange(n)})
        assert np.array_equal(got[ks], coracle.zx_coeffs(r.g, r.h, ks, r.ow)), "request %d sampled" % i
        if i % 6 == 0:
            assert np.array_equal(got, r.one_at_a_time()), "request %d vs one-at-a-time" % i
