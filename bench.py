#!/usr/bin/env python3
"""Benchmark of the cache-friendly TFT hot path on one MI355X.

Workload (one step = the whole hot path over one batch of synthetic input):
the large-coefficient Schoenhage-Strassen product in Z[x] -- two polynomials
of 50,000 coefficients of 32,000 bits, ring Z/(2^65536+1), transform length
L = 2^17 split 2^8 x 2^9, truncation n = 99,999: pack, TFT(g), TFT(h),
99,999 pointwise products, ITFT, unpack (zx_mul_ss).

Metric: TFT+ITFT throughput in GB/s of algorithmic bytes -- the cells each
transform's top-level column and row passes read and write (Alg. 1 and
Alg. 2 loop bounds, 8192 bytes per cell) -- over the time of the three
transforms, measured with HIP events on the stream the kernels run on.
Inputs are resident in HBM before the timed region.  One JSON line is printed.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
    python bench.py --split-sweep     # cache-friendly vs divide-and-conquer transforms
    python bench.py --alu-probe       # register-only issue rates behind the pointwise ceiling
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "TFT+ITFT GB/s & % HBM peak; batched Z[x] muls/s vs one-at-a-time (bit-exact)"
HBM_PEAK_GBS = 8000.0
# MI355X: 256 compute units of 4 SIMDs at 2.4 GHz; a SIMD issues one wave64
# VALU instruction per `cycles` clocks (4 for a full-rate operation)
CUS, SIMDS, CLOCK_HZ, WAVE = 256, 4, 2.4e9, 64
CPU_THREAD_CAP = 16  # worker threads the GPU host's CPU share allows


def lane_ops_peak(cycles_per_wave_instr):
    """Lane operations per second of one instruction issued back to back on every SIMD."""
    return CUS * SIMDS * CLOCK_HZ * WAVE / cycles_per_wave_instr


def cycles_per_wave_instr(lane_ops_per_s):
    """Clocks per wave64 instruction implied by a measured issue rate at 2.4 GHz."""
    return CUS * SIMDS * CLOCK_HZ * WAVE / lane_ops_per_s


def _split(l):
    return l // 2, l - l // 2


def alg_cells_tft(l, z, n):
    """Cells read + written by Alg. 1's top-level column and row passes."""
    l1, l2 = _split(l)
    L2 = 1 << l2
    n1p = -(-n // L2)
    z1, z2 = divmod(z, L2)
    z2p = L2 if z1 else z2
    return z + z2p * n1p + n1p * z2p + n


def alg_cells_itft(l, z, n, f):
    """Cells read + written by Alg. 2's top-level rows, right columns, last row and left columns."""
    l1, l2 = _split(l)
    L2 = 1 << l2
    n1, n2 = divmod(n, L2)
    z1, z2 = divmod(z, L2)
    fp = 1 if n2 + f > 0 else 0
    z2p = L2 if z1 else z2
    m, mp = min(n2, z2), max(n2, z2)
    cells = n1 * L2 * 2
    for u in range(n2, z2p):
        cells += (z1 + 1 if u < mp else z1) + n1 + fp
    if fp:
        cells += z2p + n2 + f
    for u in range(n2):
        cells += (z1 + 1 if u < m else z1) + n1 + 1
    return cells


def pointwise_limb_macs(N):
    """Limb multiply-accumulates of one pointwise product in Z/(2^N+1) as the
    library computes it: N = 16384 .. 131072 go through one more
    Schoenhage-Strassen level (64 inner products of WI x WI limbs mod
    2^(32 WI)+1, WI = 32, 64, 96, 160), other sizes are schoolbook (N/32)^2."""
    inner = {16384: 32, 32768: 64, 65536: 96, 131072: 160}.get(N)
    if inner:
        return 64 * inner * inner, ("fermat_pointwise_nested_kernel: 64 inner products of %d x %d limbs "
                                    "mod 2^%d+1 between length-64 transforms" % (inner, inner, 32 * inner))
    W = N // 32
    return W * W, "fermat_pointwise_kernel: %d x %d limbs (schoolbook)" % (W, W)


def host_threads():
    """(nproc, threads used): the CPUs this process may run on, capped at the
    GPU host's share."""
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return nproc, max(1, min(CPU_THREAD_CAP, nproc))


def cpu_baseline(g_limbs_arr, N, l, z, n, alg_bytes, budget_s=12.0, one_thread_s=3.0):
    """The oracle (eq. (1) evaluated directly, plain C) on a bounded sample, extrapolated;
    on all threads the host allows, and on one thread."""
    import numpy as np
    from oracle import coracle
    nproc, threads = host_threads()
    L = 1 << l
    W = N // 32
    a = np.zeros((z, W), dtype=np.uint32)
    a[:, : g_limbs_arr.shape[1]] = g_limbs_arr[:z]
    tops = np.zeros(z, dtype=np.uint32)
    # one probe output to size the sample (about budget_s seconds on all threads),
    # then a batch of outputs on all threads
    t0 = time.perf_counter()
    coracle.fermat_dft_sampled(N, L, 0, a, tops, [1], nthreads=1)
    t_one = time.perf_counter() - t0
    k = max(threads, min(64 * threads, int(budget_s * threads / max(t_one, 1e-6))))
    k -= k % threads
    js = [(7919 * i) % n for i in range(k)]
    t0 = time.perf_counter()
    coracle.fermat_dft_sampled(N, L, 0, a, tops, js, nthreads=threads)
    t_k = time.perf_counter() - t0
    per_output = t_k / k  # wall seconds per TFT output (z terms) with `threads` threads
    # the direct transforms: 2 TFTs of n outputs with z terms, one inverse of n outputs with n terms
    outputs = 2 * n + n * (n / z)
    total_s = per_output * outputs
    # one thread, on a smaller sample
    k1 = max(1, min(k, int(one_thread_s / max(t_one, 1e-6))))
    t0 = time.perf_counter()
    coracle.fermat_dft_sampled(N, L, 0, a, tops, js[:k1], nthreads=1)
    t_1 = time.perf_counter() - t0
    total_1 = t_1 / k1 * outputs
    return {"value": alg_bytes / total_s / 1e9, "unit": "GB/s", "cores": threads, "nproc": nproc,
            "kind": "oracle", "one_thread_value": alg_bytes / total_1 / 1e9,
            "sample": "eq. (1) evaluated directly for %d output indices of TFT(g) (%d terms each) on %d threads "
                      "(nproc %d, capped at %d), %.1f s, and for %d of them on 1 thread, %.1f s; extrapolated by "
                      "term count to TFT(g)+TFT(h)+ITFT (%.0f s on %d threads, %.0f s on 1)"
                      % (k, z, threads, nproc, CPU_THREAD_CAP, t_k, k1, t_1, total_s, threads, total_1)}


def alu_probe(T, blocks=None, iters=(16384, 8192, 4096)):
    """Register-only issue rates (tft_alu_rate) of v_add_u32, v_mad_u64_u32 and the
    two-instruction limb multiply-accumulate, and the clocks per wave instruction
    they imply at 2.4 GHz.  The multiply-accumulate rate is the ceiling of the
    pointwise kernel's inner loop."""
    blocks = blocks or CUS * 8
    out = {"blocks": blocks, "threads_per_block": 256}
    for kind, name, it in ((0, "add_u32", iters[0]), (1, "mad_u64_u32", iters[1]), (2, "mac_pair", iters[2])):
        best, hz_best = None, 0.0
        for _ in range(3):
            ms, ops, hz = T.alu_rate(kind, blocks, it)
            rate = ops / (ms * 1e-3)
            if best is None or rate > best:
                best, hz_best = rate, hz
        out[name + "_T_per_s"] = round(best / 1e12, 3)
        out[name + "_cycles_per_wave_instr"] = round(cycles_per_wave_instr(best), 2)
        out[name + "_clock_GHz"] = round(hz_best / 1e9, 3)
        if hz_best > 0:  # clocks per instruction at the clock the probe measured
            out[name + "_cycles_at_measured_clock"] = round(cycles_per_wave_instr(best) * hz_best / CLOCK_HZ, 2)
    return out


def nega_case4_transforms(T, torch, reps=5):
    """The transforms of the (Z/mZ)[x] product, 500000 x 500000 with K = 1024: two
    TFT(2^11, 977 -> 1953) and one ITFT(1953) over (Z/mZ)[y]/(y^1024+1), timed
    one by one with HIP events (median of reps), as GB/s of algorithmic bytes
    (the cells Alg. 1 / Alg. 2's top-level passes read and write, 8192 bytes each)."""
    from synth import workloads as wl
    m, _, _ = wl.zmx_operands()
    K, l, z, n = 1024, 11, 977, 1953
    ring = T.nega_ring(K, m)
    L = 1 << l
    x = torch.randint(0, 1 << 62, (L * K,), dtype=torch.int64, device="cuda") % m
    wsf = torch.empty(T.transform_workspace(ring, 0, l, 0, z, n), dtype=torch.uint8, device="cuda")
    wsi = torch.empty(T.transform_workspace(ring, 1, l, 0, n, n, 0), dtype=torch.uint8, device="cuda")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return sorted(ts)[len(ts) // 2]

    tft_ms = timed(lambda: T.tft_forward(ring, l, 0, z, n, x, wsf))
    itft_ms = timed(lambda: T.itft_inverse(ring, l, 0, n, n, 0, x, wsi))
    cells = 2 * alg_cells_tft(l, z, n) + alg_cells_itft(l, n, n, 0)
    total = 2 * tft_ms + itft_ms
    gbs = cells * 8 * K / (total * 1e-3) / 1e9
    return {"workload": "2 x TFT(2^11, z=977, n=1953) + ITFT(1953) over (Z/mZ)[y]/(y^1024+1)",
            "tft_ms": round(tft_ms, 4), "itft_ms": round(itft_ms, 4), "alg_cells": cells,
            "alg_bytes": cells * 8 * K, "gb_per_s": round(gbs, 2), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}


def _source_hash():
    """Hash of the library sources (kernels, planner, ABI): identifies the kernel version profiled."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_0810_3203_amd", "csrc", "*"))) + [
        os.path.join(ROOT, "include", "tft.h")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(path=os.path.join(ROOT, "profiles", "ss_large_L2e17_pmc_traffic.md")):
    """HBM bytes per leaf launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, if it was
    taken with the current sources (else None: the counters describe another kernel)."""
    import re
    try:
        with open(path) as fh:
            text = fh.read()
    except OSError:
        return None
    m = re.search(r"when measured: `([0-9a-f]+)` \(traffic_bytes_per_launch = (\d+)\)", text)
    if not m or m.group(1) != _source_hash():
        return None
    return int(m.group(2))


def _progress(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def _leg(fn):
    """fn(), or {"error": message} if it raises (traceback on stderr)."""
    import traceback
    try:
        return fn()
    except Exception as e:  # noqa: BLE001 - reported in the output line
        traceback.print_exc()
        return {"error": "%s: %s" % (type(e).__name__, str(e)[:400])}


def batch_leg(T, torch, count=4096, train_count=32, heldout=16, replays=3, k1_stride=16):
    """Many Z[x] products of uneven lengths in batched plans (hipGraph replay), with
    each request's parameters chosen by the learned policy: the cost model trained
    on batch-context timings of candidates (k, split, whole-row padding, twist) of
    requests outside the batch.  That is the reported number.  Two labelled
    comparisons run the same batch: the fixed rule (the default rule's k with
    whole-row padding and the twist for every request) and the cost model
    trained on single-product timings.  All against one-at-a-time zx_mul_ss with
    the default rule; outputs compared bit for bit on the device."""
    from paper_0810_3203_amd import tuning
    from synth import device as dev

    t0 = time.perf_counter()
    ops = [dev.batch_request(torch, i, "cuda") for i in range(count)]
    outs_b, outs_s, reqs = [], [], []
    for g, h in ops:
        ow = (32 * (g.shape[1] + h.shape[1]) + (min(g.shape[0], h.shape[0]) - 1).bit_length() + 31) // 32
        ob = torch.empty((g.shape[0] + h.shape[0] - 1, ow), dtype=torch.int32, device="cuda")
        outs_b.append(ob)
        outs_s.append(torch.empty_like(ob))
        reqs.append(T.zx_request(g, h, ob))
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    _progress("batch: %d requests generated in %.1f s" % (count, gen_s))

    # cost model: exhaustive timings of requests outside the batch, then training
    t0 = time.perf_counter()
    extra = [dev.batch_request(torch, 100000 + i, "cuda") for i in range(train_count + heldout)]
    ereq, keep = [], []
    for g, h in extra:
        ow = (32 * (g.shape[1] + h.shape[1]) + (min(g.shape[0], h.shape[0]) - 1).bit_length() + 31) // 32
        o = torch.empty((g.shape[0] + h.shape[0] - 1, ow), dtype=torch.int32, device="cuda")
        keep.append(o)
        ereq.append(T.zx_request(g, h, o))
    tim = tuning.time_candidates(ereq[:train_count], reps=3)
    X, y = tuning.training_rows(ereq[:train_count], tim)
    tune_s = time.perf_counter() - t0
    _progress("batch: %d training requests timed in %.1f s" % (train_count, tune_s))
    t0 = time.perf_counter()
    model, loss = tuning.train_model(X, y, iters=3000)
    train_s = time.perf_counter() - t0
    ho = tuning.time_candidates(ereq[train_count:], reps=3)
    rows = tuning.policy_times(ereq[train_count:], ho, model)
    t_best = sum(r["best"] for r in rows)
    t_mlp = sum(r["mlp"] for r in rows)
    t_def = sum(r["default"] for r in rows)
    _progress("batch: model trained (loss %.4f), held-out regret %.3f" % (loss, t_mlp / t_best - 1))
    # the same model trained on batch-context timings (copies of a request in one plan)
    t0 = time.perf_counter()
    tim_b = tuning.time_candidates_in_batch(ereq[:train_count])
    Xb, yb = tuning.training_rows(ereq[:train_count], tim_b)
    model_b, loss_b = tuning.train_model(Xb, yb, iters=3000)
    ho_b = tuning.time_candidates_in_batch(ereq[train_count:])
    rows_b = tuning.policy_times(ereq[train_count:], ho_b, model_b)
    tb_best, tb_mlp, tb_def = (sum(r[k] for r in rows_b) for k in ("best", "mlp", "default"))
    tune_b_s = time.perf_counter() - t0
    del keep, extra, ereq
    _progress("batch: batch-context model trained (loss %.4f), held-out regret %.3f, %.1f s"
              % (loss_b, tb_mlp / tb_best - 1, tune_b_s))

    # the learned policy: the batch-context model's choice per request
    arr = T.requests_array(reqs)
    t0 = time.perf_counter()
    model_b.choose(arr)
    choose_s = time.perf_counter() - t0
    ks = {}
    for r in arr:
        ks[r.params.k] = ks.get(r.params.k, 0) + 1
    padded = sum(1 for r in arr if r.params.pad_rows)
    twisted = sum(1 for r in arr if r.params.zeta_exp)

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_plan(req_arr, label):
        t0 = time.perf_counter()
        plan = T.BatchPlan(req_arr, max_workspace=96 << 30)
        build_s = time.perf_counter() - t0
        assert all(s == 0 for s in plan.status())
        ws = torch.empty(plan.workspace, dtype=torch.uint8, device="cuda")
        plan.execute(ws, use_graph=True)  # direct run + capture
        plan.execute(ws, use_graph=True)  # first replay
        torch.cuda.synchronize()
        e0.record()
        for _ in range(replays):
            plan.execute(ws, use_graph=True)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / replays
        _progress("batch (%s): graph replay %.1f ms (%d launches)" % (label, ms, plan.launches))
        n_launch = plan.launches
        plan.close()
        del ws
        return ms, n_launch, build_s

    batch_ms, launches, plan_s = time_plan(arr, "learned")

    # one at a time, default rule, no graph
    params = [T.ss_default_params(g.shape[0], g.shape[1], h.shape[0], h.shape[1]) for g, h in ops]
    need = max(T.zx_mul_ss_workspace(g.shape[0], g.shape[1], h.shape[0], h.shape[1], p)
               for (g, h), p in zip(ops, params))
    ws1 = torch.empty(need, dtype=torch.uint8, device="cuda")

    def one_pass(sel, par, outs):
        for i in sel:
            g, h = ops[i]
            T.zx_mul_ss(g, h, outs[i], par[i], ws=ws1)

    one_pass(range(count), params, outs_s)  # builds and uploads every shape's plans
    torch.cuda.synchronize()
    e0.record()
    one_pass(range(count), params, outs_s)
    e1.record()
    torch.cuda.synchronize()
    single_ms = e0.elapsed_time(e1)
    _progress("batch: one at a time %.1f ms" % single_ms)
    exact = all(torch.equal(a, b) for a, b in zip(outs_b, outs_s))

    # comparison 1: the fixed rule, the default rule's k with whole-row padding
    # and the forward twist theta^(3N/2) for every request (the options merged
    # passes reward); N from the ring-size feature log2(W)/12
    arr2 = T.requests_array(reqs)
    for r in arr2:
        r.params = tuning.rule_params(r)
    batch_ms_rule, launches_rule, _ = time_plan(arr2, "fixed rule")
    exact_rule = all(torch.equal(a, b) for a, b in zip(outs_b, outs_s))
    # comparison 2: the cost model trained on single-product timings
    arr3 = T.requests_array(reqs)
    model.choose(arr3)
    batch_ms_single, launches_single, _ = time_plan(arr3, "single-product cost model")
    exact_single = all(torch.equal(a, b) for a, b in zip(outs_b, outs_s))

    # the paper's literal product (k = 1) one at a time, on every k1_stride-th request
    p1 = [T.SSParams(0, 0, T.Split(0, 0), 1)] * count
    sel = list(range(0, count, k1_stride))
    need1 = max(T.zx_mul_ss_workspace(ops[i][0].shape[0], ops[i][0].shape[1], ops[i][1].shape[0],
                                      ops[i][1].shape[1], p1[i]) for i in sel)
    del ws1
    ws1 = torch.empty(need1, dtype=torch.uint8, device="cuda")
    one_pass(sel, p1, outs_s)
    torch.cuda.synchronize()
    e0.record()
    one_pass(sel, p1, outs_s)
    e1.record()
    torch.cuda.synchronize()
    k1_ms = e0.elapsed_time(e1) * count / len(sel)
    exact_k1 = all(torch.equal(outs_b[i], outs_s[i]) for i in sel)
    del ws1

    muls = count / (batch_ms * 1e-3)
    return {
        "workload": "%d Z[x] products, lengths uniform in [100, 20000], 1000-bit coefficients" % count,
        "policy": "learned: cost model trained on batch-context timings, argmin per request",
        "muls_per_s": round(muls, 1),
        "batch_ms": round(batch_ms, 3),
        "launches": launches,
        "one_at_a_time_muls_per_s": round(count / (single_ms * 1e-3), 1),
        "one_at_a_time_ms": round(single_ms, 3),
        "speedup_vs_one_at_a_time": round(single_ms / batch_ms, 3),
        "k1_one_at_a_time_ms_extrapolated": round(k1_ms, 3),
        "speedup_vs_k1_one_at_a_time": round(k1_ms / batch_ms, 3),
        "k1_sample": "every %dth request (%d), time scaled by %d/%d" % (k1_stride, len(sel), count, len(sel)),
        "bit_exact_vs_one_at_a_time": bool(exact and exact_k1 and exact_rule and exact_single),
        "comparison_fixed_rule": {"batch_ms": round(batch_ms_rule, 3), "launches": launches_rule,
                                  "speedup_vs_one_at_a_time": round(single_ms / batch_ms_rule, 3),
                                  "learned_gain": round(batch_ms_rule / batch_ms, 4)},
        "comparison_single_product_cost_model": {"batch_ms": round(batch_ms_single, 3), "launches": launches_single,
                                                 "learned_gain": round(batch_ms_single / batch_ms, 4)},
        "learned_model": {"train_requests": train_count, "train_rows": len(Xb), "final_loss": round(loss_b, 5),
                          "heldout_requests": heldout, "heldout_regret": round(tb_mlp / tb_best - 1, 4),
                          "heldout_gain_vs_default": round(tb_def / tb_mlp, 4), "host_s": round(tune_b_s, 2)},
        "k_chosen": {str(k): v for k, v in sorted(ks.items())},
        "padded_chosen": padded,
        "twisted_chosen": twisted,
        "single_product_cost_model": {"train_rows": len(X), "final_loss": round(loss, 5),
                                      "heldout_regret": round(t_mlp / t_best - 1, 4),
                                      "heldout_gain_vs_default": round(t_def / t_mlp, 4)},
        "host_s": {"generate": round(gen_s, 2), "tune": round(tune_s, 2), "train": round(train_s, 2),
                   "choose": round(choose_s, 2), "plan": round(plan_s, 2)},
    }


def other_products(T, torch, reps=5):
    """Latency of the other product workloads (median of `reps` runs, HIP events on the stream):
    Z[x] 500 x 500 of 64 bits (ring 2^512+1, L = 2^10) and 3000 x 3000 of 2000 bits (2^4096+1, L = 2^13),
    both latency-bound and reported against their launch floor (launches x one back-to-back launch),
    and the Schoenhage-Nussbaumer product in (Z/mZ)[x], 500000 x 500000, K = 1024."""
    import numpy as np
    from synth import workloads as wl

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return sorted(ts)[len(ts) // 2]

    # the floor of a launch-bound product: its kernel launches (pack of g and h,
    # the leaf passes, the pointwise products, unpack) times the time of one
    # back-to-back launch of a trivial kernel on the same stream
    one = torch.zeros(1, device="cuda")
    one.add_(1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(200):
        one.add_(1)
    e1.record()
    torch.cuda.synchronize()
    launch_ms = e0.elapsed_time(e1) / 200
    out = {"launch_ms": round(launch_ms, 5)}
    for c in (1, 2):
        g, h = wl.zx_operands(c)
        dg = torch.from_numpy(g.view(np.int32)).cuda()
        dh = torch.from_numpy(h.view(np.int32)).cuda()
        ow = (32 * (g.shape[1] + h.shape[1]) + (min(g.shape[0], h.shape[0]) - 1).bit_length() + 31) // 32
        o = torch.empty((g.shape[0] + h.shape[0] - 1, ow), dtype=torch.int32, device="cuda")
        ws = torch.empty(T.zx_mul_ss_workspace(g.shape[0], g.shape[1], h.shape[0], h.shape[1]), dtype=torch.uint8,
                         device="cuda")
        ms = timed(lambda: T.zx_mul_ss(dg, dh, o, ws=ws))
        launches = T.zx_mul_ss_timed(dg, dh, o, ws=ws)["leaf_launches"] + 4
        out["zx_%dx%d_%dbit" % (g.shape[0], h.shape[0], wl.ZX_CASES[c]["bits"])] = {
            "ms": round(ms, 4), "launches": launches, "launch_floor_ms": round(launches * launch_ms, 4),
            "frac_of_launch_floor": round(launches * launch_ms / ms, 3)}
    m, g, h = wl.zmx_operands()
    dg = torch.from_numpy(g.view(np.int64)).cuda()
    dh = torch.from_numpy(h.view(np.int64)).cuda()
    o = torch.empty(len(g) + len(h) - 1, dtype=torch.int64, device="cuda")
    ws = torch.empty(T.zmx_mul_nussbaumer_workspace(len(g), len(h), 10), dtype=torch.uint8, device="cuda")
    out["zmx_500000x500000_K1024_ms"] = round(timed(lambda: T.zmx_mul_nussbaumer(dg, dh, m, 10, o, ws=ws)), 3)
    return out


def prime_leg(T, torch, lg=1 << 23, lh=1 << 23, reps=5):
    """The small-coefficient case (Sect. 6): the product of two polynomials of
    2^23 coefficients in (Z/pZ)[x], p = 15 2^27 + 1 (n = 2^24 - 1, L = 2^24).
    The two TFTs and the ITFT are timed one by one as plans made beforehand
    (descriptors already in device memory; HIP events, median of reps) and
    reported as algorithmic GB/s: the cells Alg. 1 / Alg. 2's top-level passes
    read and write, 4 bytes each.  tft_forward, which also copies the plan's
    descriptors to the device on every call, is timed beside them.  The whole
    product through zpx_mul_ntt, with and without Sect. 6's whole-row padding,
    is timed the same way; its output must not change with padding."""
    import numpy as np
    ring = T.prime_ring()
    n = lg + lh - 1
    l = max(1, (n - 1).bit_length())
    L = 1 << l
    rng = np.random.default_rng(6)
    g = torch.from_numpy(rng.integers(0, T.PRIME_P, size=lg, dtype=np.uint64).astype(np.uint32).view(np.int32)).cuda()
    h = torch.from_numpy(rng.integers(0, T.PRIME_P, size=lh, dtype=np.uint64).astype(np.uint32).view(np.int32)).cuda()
    A = torch.zeros(L, dtype=torch.int32, device="cuda")
    wsf = torch.empty(T.transform_workspace(ring, 0, l, 0, lg, n), dtype=torch.uint8, device="cuda")
    pf = T.Plan(ring, 0, l, 0, lg, n)
    pi = T.Plan(ring, 1, l, 0, n, n, 0)

    def timed(fn, prep=None):
        if prep:
            prep()
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            if prep:
                prep()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return sorted(ts)[len(ts) // 2]

    tft_ms = timed(lambda: pf.execute(A), prep=lambda: A[:lg].copy_(g))
    itft_ms = timed(lambda: pi.execute(A))
    one_call_ms = timed(lambda: T.tft_forward(ring, l, 0, lg, n, A, wsf), prep=lambda: A[:lg].copy_(g))
    cells = 2 * alg_cells_tft(l, lg, n) + alg_cells_itft(l, n, n, 0)
    total = 2 * tft_ms + itft_ms
    gbs = cells * 4 / (total * 1e-3) / 1e9
    out0 = torch.empty(n, dtype=torch.int32, device="cuda")
    out1 = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = torch.empty(2 * L * 4, dtype=torch.uint8, device="cuda")
    prod_ms = timed(lambda: T.zpx_mul_ntt(g, h, out0, 0, ws))
    prod_pad_ms = timed(lambda: T.zpx_mul_ntt(g, h, out1, 1, ws))
    exp = pf.export()
    return {"workload": "(Z/pZ)[x] product, p = 15 2^27 + 1: %d x %d coefficients, L = 2^%d, n = %d" % (lg, lh, l, n),
            "tft_passes": len(exp["passes"]), "tft_ms": round(tft_ms, 4), "itft_ms": round(itft_ms, 4),
            "tft_forward_call_ms": round(one_call_ms, 4), "alg_cells": cells, "alg_bytes": cells * 4,
            "transforms_gb_per_s": round(gbs, 2), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
            "product_ms": round(prod_ms, 4), "product_whole_rows_ms": round(prod_pad_ms, 4),
            "whole_rows_same_output": bool(torch.equal(out0, out1))}


def padded_leg(T, torch, dg, dh, out, l, n, N, reps=3):
    """The same product with n rounded up to whole rows of the paper split
    (Sect. 6 zero-padding: no partial last row in the ITFT), with the forward
    twist zeta = theta^(3N/2) (the ITFT then takes zeta^2), and with both; every
    output must equal the plain one bit for bit."""
    L2 = 1 << (l - l // 2)
    res = {"n_padded": -(-n // L2) * L2, "zeta_exp": 3 * N // 2}
    for name, pad, zexp in (("padded", 1, 0), ("twisted", 0, 3 * N // 2), ("padded_twisted", 1, 3 * N // 2)):
        p = T.SSParams(0, 0, T.Split(0, 0), 1, pad, zexp)
        ws = torch.empty(T.zx_mul_ss_workspace(dg.shape[0], dg.shape[1], dh.shape[0], dh.shape[1], p),
                         dtype=torch.uint8, device="cuda")
        o = torch.empty_like(out)
        T.zx_mul_ss_timed(dg, dh, o, p, ws=ws)
        runs = sorted((T.zx_mul_ss_timed(dg, dh, o, p, ws=ws) for _ in range(reps)), key=lambda t: t["total_ms"])
        t = runs[len(runs) // 2]
        res[name] = {"total_ms": round(t["total_ms"], 3),
                     "transform_ms": round(t["tft_g_ms"] + t["tft_h_ms"] + t["itft_ms"], 3),
                     "tft_ms": round(t["tft_g_ms"] + t["tft_h_ms"], 3), "itft_ms": round(t["itft_ms"], 3),
                     "leaf_launches": t["leaf_launches"], "same_output": bool(torch.equal(o, out))}
        del ws, o
    return res


def split_sweep(T, torch, bits=8000, lo=512, hi=16384, step=1.05, reps=3):
    """Cache-friendly against divide-and-conquer transforms (Sect. 1, Sect. 5.1
    experiment shape): Z[x] products of two random `bits`-bit polynomials of equal
    length, lengths lo..hi in 5% steps, one coefficient per ring element.  All
    runs use the same ring, length and leaf size; the divide-and-conquer run
    splits L1 = 2 at every level above the leaf, and a third run pads n to whole
    rows of the paper split (Sect. 6).  Median of `reps` runs each; the outputs
    are compared bit for bit."""
    import numpy as np
    from synth import workloads as wl
    from synth.splitmix import SplitMix64

    limbs = bits // 32
    lens, x = [], float(lo)
    while round(x) <= hi:
        lens.append(int(round(x)))
        x *= step
    rng = SplitMix64(0x0810320300000006)
    rows = []
    for ln in lens:
        g, h = wl.random_ints(rng, ln, bits), wl.random_ints(rng, ln, bits)
        dg = torch.from_numpy(g.view(np.int32)).cuda()
        dh = torch.from_numpy(h.view(np.int32)).cuda()
        ow = (32 * 2 * limbs + (ln - 1).bit_length() + 31) // 32
        res = {}
        outs = []
        for name, top, pad, zexp in (("bailey", 0, 0, 0), ("dc", T.SPLIT_DC, 0, 0), ("padded", 0, 1, 0),
                                     ("padded_twisted", 0, 1, 3 * 16384 // 2)):
            p = T.SSParams(0, 0, T.Split(top, 0), 1, pad, zexp)
            ws = torch.empty(T.zx_mul_ss_workspace(ln, limbs, ln, limbs, p), dtype=torch.uint8, device="cuda")
            o = torch.empty((2 * ln - 1, ow), dtype=torch.int32, device="cuda")
            T.zx_mul_ss_timed(dg, dh, o, p, ws=ws)
            runs = sorted((T.zx_mul_ss_timed(dg, dh, o, p, ws=ws) for _ in range(reps)), key=lambda t: t["total_ms"])
            t = runs[len(runs) // 2]
            res[name] = t
            outs.append(o)
            del ws
        same = all(bool(torch.equal(outs[0], o)) for o in outs[1:])
        b, d, w, wt = res["bailey"], res["dc"], res["padded"], res["padded_twisted"]

        def tr(t):
            return t["tft_g_ms"] + t["tft_h_ms"] + t["itft_ms"]

        rows.append({"len": ln, "N": b["N"], "l": b["l"], "bailey_ms": round(b["total_ms"], 4),
                     "dc_ms": round(d["total_ms"], 4), "bailey_transform_ms": round(tr(b), 4),
                     "dc_transform_ms": round(tr(d), 4), "bailey_launches": b["leaf_launches"],
                     "dc_launches": d["leaf_launches"], "padded_ms": round(w["total_ms"], 4),
                     "padded_transform_ms": round(tr(w), 4), "padded_launches": w["leaf_launches"],
                     "padded_twisted_ms": round(wt["total_ms"], 4), "padded_twisted_transform_ms": round(tr(wt), 4),
                     "same_output": same})
        _progress("split sweep len %d: bailey %.3f ms, dc %.3f ms, padded %.3f ms, same %s"
                  % (ln, b["total_ms"], d["total_ms"], w["total_ms"], same))
        del outs, dg, dh

    def spread(key, ref):
        v = sorted(r[key] / r[ref] for r in rows)
        return {"min": round(v[0], 3), "median": round(v[len(v) // 2], 3), "max": round(v[-1], 3)}

    return {"experiment": "Z[x] products, %d-bit coefficients, lengths %d..%d in %d%% steps: "
                          "cache-friendly (paper split) vs divide-and-conquer transforms vs "
                          "whole-row padding" % (bits, lo, hi,
                                                                                            round(100 * (step - 1))),
            "rows": rows, "all_outputs_equal": all(r["same_output"] for r in rows),
            "product_time_ratio_dc_over_bailey": spread("dc_ms", "bailey_ms"),
            "transform_time_ratio_dc_over_bailey": spread("dc_transform_ms", "bailey_transform_ms"),
            "product_time_ratio_padded_over_bailey": spread("padded_ms", "bailey_ms"),
            "transform_time_ratio_padded_over_bailey": spread("padded_transform_ms", "bailey_transform_ms"),
            "product_time_ratio_padded_twisted_over_bailey": spread("padded_twisted_ms", "bailey_ms"),
            "transform_time_ratio_padded_twisted_over_bailey": spread("padded_twisted_transform_ms",
                                                                      "bailey_transform_ms")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-products measurement")
    ap.add_argument("--no-padded", action="store_true",
                    help="skip the padded and twisted runs of the large product (profiles of the plain one)")
    ap.add_argument("--split-sweep", action="store_true",
                    help="instead of the benchmark: cache-friendly vs divide-and-conquer transforms over a sweep "
                         "of Z[x] products with 8000-bit coefficients (one JSON line)")
    ap.add_argument("--large-only", action="store_true",
                    help="only the large product (for profiler runs): no probe, other products or batch")
    ap.add_argument("--batch-only", action="store_true",
                    help="instead of the benchmark: only the batched-products leg (one JSON line)")
    ap.add_argument("--prime-only", action="store_true",
                    help="instead of the benchmark: only the (Z/pZ)[x] small-coefficient leg (one JSON line)")
    ap.add_argument("--alu-probe", action="store_true",
                    help="instead of the benchmark: only the register-only issue-rate probe (one JSON line)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run three plain 1 GiB device copies (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (--gpus %d refused)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_0810_3203_amd as T
    from synth import workloads as wl

    torch.cuda.set_device(0)
    if args.split_sweep:
        print(json.dumps(split_sweep(T, torch)), flush=True)
        return
    if args.alu_probe:
        print(json.dumps(alu_probe(T)), flush=True)
        return
    if args.batch_only:
        print(json.dumps(batch_leg(T, torch)), flush=True)
        return
    if args.prime_only:
        print(json.dumps(prime_leg(T, torch)), flush=True)
        return
    spec = wl.ZX_CASES[3]
    g, h = wl.zx_operands(3)
    len_g, len_h = g.shape[0], h.shape[0]
    n = len_g + len_h - 1
    N, l = spec["N"], spec["l"]
    out_limbs = (32 * (g.shape[1] + h.shape[1]) + (min(len_g, len_h) - 1).bit_length() + 31) // 32
    dg = torch.from_numpy(g.view(np.int32)).cuda()
    dh = torch.from_numpy(h.view(np.int32)).cuda()
    out = torch.empty((n, out_limbs), dtype=torch.int32, device="cuda")
    ws = torch.empty(T.zx_mul_ss_workspace(len_g, g.shape[1], len_h, h.shape[1]), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()

    cell_bytes = N // 8
    cells = alg_cells_tft(l, len_g, n) + alg_cells_tft(l, len_h, n) + alg_cells_itft(l, n, n, 0)
    alg_bytes = cells * cell_bytes

    _progress("large product: warmup")
    for _ in range(args.warmup):
        T.zx_mul_ss_timed(dg, dh, out, ws=ws)
    torch.cuda.synchronize()
    phases = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        phases.append(T.zx_mul_ss_timed(dg, dh, out, ws=ws))
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1000.0 / args.steps

    def avg(key):
        return sum(p[key] for p in phases) / len(phases)

    transform_ms = avg("tft_g_ms") + avg("tft_h_ms") + avg("itft_ms")
    leaf_ms = avg("leaf_kernel_ms")
    launches = phases[0]["leaf_launches"]
    value = alg_bytes / (transform_ms * 1e-3) / 1e9
    achieved = alg_bytes / (leaf_ms * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "Z[x] product by Schoenhage-Strassen: 50000 x 50000 coefficients of 32000 bits, "
                        "R = Z/(2^65536+1), L = 2^17 (2^8 x 2^9), n = 99999",
            "alg_cells": cells,
            "alg_bytes": alg_bytes,
            "phases_ms": {k: round(avg(k), 3) for k in ("pack_ms", "tft_g_ms", "tft_h_ms", "pointwise_ms",
                                                         "itft_ms", "unpack_ms", "total_ms")},
            "transform_ms": round(transform_ms, 3),
            "pct_hbm_peak": round(100.0 * value / HBM_PEAK_GBS, 2),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": profiled_traffic(),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "alg_bytes_per_launch": int(alg_bytes / max(1, launches)),
            "kernel": "fermat_leaf2_kernel<32,true> (%d launches per step)" % launches,
            "avg_launch_ms": round(leaf_ms / max(1, launches), 4),
        },
    }
    # the pointwise stage's multiplications are limb multiply-accumulates
    # (v_mad_u64_u32 + v_addc_co_u32); their ceiling is that pair's
    # register-only issue rate.  At N = 65536 a product is 64 inner products of
    # 96 x 96 limbs mod 2^3072+1 between two length-64 transforms (one more
    # Schoenhage-Strassen level); the rate counts those multiply-accumulates,
    # and the schoolbook count the same stage replaces is reported beside it.
    probe = {} if args.large_only else _leg(lambda: alu_probe(T))
    line["alu_probe"] = probe
    mac_peak = probe.get("mac_pair_T_per_s")
    macs, how = pointwise_limb_macs(N)
    pw_s = avg("pointwise_ms") * 1e-3
    pw_achieved = n * macs / pw_s / 1e12
    line["pointwise_roofline"] = {
        "bound": "alu",
        "achieved": round(pw_achieved, 3),
        "peak": mac_peak,
        "unit": "T limb multiply-accumulates/s",
        "frac": round(pw_achieved / mac_peak, 4) if mac_peak else None,
        "peak_source": "alu_probe.mac_pair_T_per_s (register-only loop of the same two instructions)",
        "kernel": "%d products: %s" % (n, how),
        "limb_macs_per_product": macs,
        "schoolbook_limb_macs_per_product": (N // 32) ** 2,
        "schoolbook_equivalent_T_per_s": round(n * (N // 32) ** 2 / pw_s / 1e12, 3),
    }
    if not args.no_padded:
        line["product_variants"] = _leg(lambda: padded_leg(T, torch, dg, dh, out, l, n, N, reps=3))
    del out, ws, dg, dh
    torch.cuda.empty_cache()
    # a failing secondary leg is reported in the line (with its traceback on
    # stderr) instead of taking the measured headline with it
    if not args.large_only:
        _progress("other products")
        line["other_products"] = _leg(lambda: other_products(T, torch))
        _progress("(Z/mZ)[x] product transforms")
        line["nega_case4_transforms"] = _leg(lambda: nega_case4_transforms(T, torch))
        _progress("(Z/pZ)[x] product (small coefficients)")
        line["prime_small_coefficients"] = _leg(lambda: prime_leg(T, torch))
    if not args.no_batch and not args.large_only:
        line["batch"] = _leg(lambda: batch_leg(T, torch))
    if not args.no_cpu_baseline and not args.large_only:
        _progress("cpu baseline (oracle sample)")
        line["cpu_baseline"] = cpu_baseline(g, N, l, len_g, n, alg_bytes)
    print(json.dumps(line), flush=True)
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
