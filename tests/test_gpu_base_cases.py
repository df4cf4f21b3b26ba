"""On-device check of the transform kernel's base cases (tft_debug_base_cases).

Every L = 2 base case of Alg. 1 and Alg. 2 runs on one wavefront exactly as
inside the leaf kernel, on operands of every shape in tests/base_case_defs.py
(random, 0, 1, 2^N, 2^N - 1, half-filled, whole lane chunks of zeros or ones,
single limbs, runs of ones), with boundary and random exponents, for elements
of 256 to 2048 limbs; each result must equal the base case's definition.
"""

import numpy as np
import pytest

from tests.base_case_defs import cases, expect
from tests.gpu_util import note

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0810_3203_amd as T  # noqa: E402


def _limbs(v, W):
    return np.frombuffer((v & ((1 << (32 * W)) - 1)).to_bytes(4 * W, "little"), dtype=np.uint32)


@pytest.mark.parametrize("N,count", [(8192, 600), (16384, 400), (32768, 300), (65536, 300)])
def test_base_cases_on_device(N, count):
    W = N // 32
    cs = cases(N, count, seed=N + count)
    rec = 4 + 2 * W
    buf = np.zeros((count, rec), dtype=np.uint32)
    for i, (code, s, x0, x1) in enumerate(cs):
        buf[i, 0], buf[i, 1] = code, s
        buf[i, 2], buf[i, 3] = x0 >> N, x1 >> N
        buf[i, 4:4 + W] = _limbs(x0, W)
        buf[i, 4 + W:] = _limbs(x1, W)
    note("base cases on device N=%d, %d cases" % (N, count))
    din = torch.from_numpy(buf.reshape(-1).view(np.int32)).cuda()
    dout = torch.zeros_like(din)
    T.debug_base_cases(T.fermat_ring(N), count, din, dout)
    torch.cuda.synchronize()
    out = dout.cpu().numpy().view(np.uint32).reshape(count, rec)
    bad = []
    for i, (code, s, x0, x1) in enumerate(cs):
        y0 = int.from_bytes(out[i, 4:4 + W].tobytes(), "little") + (int(out[i, 2]) << N)
        y1 = int.from_bytes(out[i, 4 + W:].tobytes(), "little") + (int(out[i, 3]) << N)
        e0, e1 = expect(code, N, s, x0, x1)
        ok = y0 == e0 and (e1 is None or y1 == e1)
        ok = ok and all(v >> N == 0 or v == 1 << N for v in (y0, y1))
        if not ok:
            bad.append(i)
    if bad:
        np.save("gpurun_out/base_case_fail_N%d.npy" % N, buf[bad[:20]]) if __import__("os").path.isdir(
            "gpurun_out") else None
    assert not bad, "%d of %d base cases wrong; first (code, s): %s" % (
        len(bad), count, [(cs[i][0], cs[i][1]) for i in bad[:10]])
