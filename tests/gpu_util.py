"""Test helpers: move cell arrays between Python/numpy values and device tensors.

Layout only (see include/tft.h): a Fermat cell array of capacity C is C*W
uint32 limbs followed by C uint32 top words; a nega cell array is C*K uint64.
Nothing here computes any part of the method.
"""

import sys

import numpy as np


def note(*args):
    """Name the GPU case about to run (flushed, so a crash still shows it)."""
    print("[gpu]", *args, flush=True)
    sys.stdout.flush()


def fermat_to_device(vals, N, cap, torch):
    """Python ints in [0, 2^N] (len <= cap) -> int32 device tensor holding the cell array."""
    W = N // 32
    arr = np.zeros(cap * (W + 1), dtype=np.uint32)
    limbs = arr[: cap * W].reshape(cap, W)
    tops = arr[cap * W:]
    for i, v in enumerate(vals):
        v = int(v)
        if v >> N:
            assert v == 1 << N
            tops[i] = 1
        else:
            limbs[i] = np.frombuffer(v.to_bytes(4 * W, "little"), dtype=np.uint32)
    return torch.from_numpy(arr.view(np.int32)).cuda()


def fermat_cells_to_device(limbs, tops, cap, torch, fill_seed=None):
    """(count, W) limbs + (count,) tops -> device cell array of capacity cap; other cells random."""
    count, W = limbs.shape
    rng = np.random.default_rng(fill_seed if fill_seed is not None else 1)
    arr = rng.integers(0, 1 << 32, size=cap * (W + 1), dtype=np.uint64).astype(np.uint32)
    arr[cap * W:] = rng.integers(0, 2, size=cap, dtype=np.uint32)  # garbage tops too
    arr[: count * W] = np.ascontiguousarray(limbs, dtype=np.uint32).reshape(-1)
    arr[cap * W: cap * W + count] = tops
    return torch.from_numpy(arr.view(np.int32)).cuda()


def fermat_from_device(t, N, cap, count):
    """First ``count`` cells of a device cell array -> (limbs (count, W) uint32, tops (count,))."""
    W = N // 32
    arr = t.cpu().numpy().view(np.uint32)
    limbs = arr[: cap * W].reshape(cap, W)[:count].copy()
    tops = arr[cap * W: cap * W + count].copy()
    return limbs, tops


def fermat_values(limbs, tops):
    N = 32 * limbs.shape[1]
    return [int.from_bytes(limbs[i].tobytes(), "little") + (int(tops[i]) << N) for i in range(limbs.shape[0])]


def nega_to_device(rows, K, cap, torch, fill=None):
    arr = np.zeros((cap, K), dtype=np.uint64) if fill is None else fill.copy()
    for i, r in enumerate(rows):
        arr[i] = np.array([int(v) for v in r], dtype=np.uint64)
    return torch.from_numpy(arr.reshape(-1).view(np.int64)).cuda()


def nega_from_device(t, K, count):
    arr = t.cpu().numpy().view(np.uint64).reshape(-1, K)
    return [tuple(int(v) for v in arr[i]) for i in range(count)]


def u32_to_device(a, torch):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def u64_to_device(a, torch):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()
