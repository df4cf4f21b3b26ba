"""Host orchestration of parameter selection for batches of Z[x] products.

Gathers exhaustive timings (tft_ss_time) of every candidate of a set of
requests, turns them into training rows for the cost model (features from
tft_ss_features, target = log of the median time in ms relative to the
request's other candidates), and applies the
three selection policies: the fixed default rule, the exhaustive best per
request, and the cost model's argmin.  The timing, training and inference all
run in libtft.so; this module only loops and marshals.
"""

import math

from . import _binding as B


def _ws_for(cands, req, torch, device):
    need = max(B.zx_mul_ss_workspace(req.len_g, req.g_limbs, req.len_h, req.h_limbs, c) for c in cands)
    return torch.empty(need, dtype=torch.uint8, device=device)


def time_candidates(reqs, reps=3, device="cuda", stream=None):
    """For each ZXRequest: (candidates, median ms per candidate, index of the fastest)."""
    import torch
    out = []
    for r in reqs:
        cands = B.ss_candidates(r.len_g, r.g_limbs, r.len_h, r.h_limbs)
        ws = _ws_for(cands, r, torch, device)
        ms, best = B.ss_time(r, cands, reps, ws, stream)
        out.append((cands, ms, best))
        del ws
    return out


def time_candidates_in_batch(reqs, copies=8, replays=2, device="cuda"):
    """Like time_candidates, but each candidate is timed where a batch runs it: a
    batch plan of `copies` copies of the request (own outputs each), replayed as a
    graph; the time per product is the replay time divided by `copies`.  Merged
    passes hide launch and tail costs that dominate single products, so these
    times rank candidates for batch plans."""
    import torch
    out = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def plan_ms(r, c, outs, n):
        arr = (B.ZXRequest * n)()
        for i in range(n):
            q = B.ZXRequest(r.g, r.len_g, r.g_limbs, r.h, r.len_h, r.h_limbs, outs[i].data_ptr(), r.out_limbs)
            q.params = c
            arr[i] = q
        plan = B.BatchPlan(arr)
        ws = torch.empty(max(1, plan.workspace), dtype=torch.uint8, device=device)
        plan.execute(ws, use_graph=True)  # direct run + capture
        plan.execute(ws, use_graph=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(replays):
            plan.execute(ws, use_graph=True)
        e1.record()
        torch.cuda.synchronize()
        plan.close()
        del ws
        return e0.elapsed_time(e1) / replays

    for r in reqs:
        cands = B.ss_candidates(r.len_g, r.g_limbs, r.len_h, r.h_limbs)
        n_out = (r.len_g + r.len_h - 1) * r.out_limbs
        outs = [torch.empty(n_out, dtype=torch.int32, device=device) for _ in range(copies)]
        ms = []
        for c in cands:
            ms.append(plan_ms(r, c, outs, copies) / copies)
        best = min(range(len(ms)), key=lambda i: (ms[i], i))
        out.append((cands, ms, best))
        del outs
    return out


def rule_params(r):
    """The fixed batch rule for one request: the default rule's k with whole-row
    padding and the forward twist theta^(3N/2) (N from the ring-size feature
    log2(W)/12), the options merged passes reward."""
    p = B.ss_default_params(r.len_g, r.g_limbs, r.len_h, r.h_limbs)
    p.pad_rows = 1
    W = int(round(2 ** (12 * B.ss_features(r.len_g, r.g_limbs, r.len_h, r.h_limbs, p)[5])))
    p.zeta_exp = 3 * (32 * W) // 2
    return p


def training_rows(reqs, timings):
    """Features (rows x SS_FEATURES) and targets from time_candidates output.  A
    target is log(ms) less the mean log(ms) over the request's candidates: only
    the order of one request's candidates decides the choice, so the model is
    fitted to that and not to the size of the request."""
    X, y = [], []
    for r, (cands, ms, _) in zip(reqs, timings):
        logs = [math.log(max(t, 1e-4)) for t in ms]
        mean = sum(logs) / len(logs)
        for c, v in zip(cands, logs):
            X.append(B.ss_features(r.len_g, r.g_limbs, r.len_h, r.h_limbs, c))
            y.append(v - mean)
    return X, y


def train_model(X, y, hidden=64, depth=3, iters=3000, lr=2e-3, seed=11, device="cuda"):
    """A new MLP trained full-batch with Adam; returns (model, final loss)."""
    import torch
    m = B.MLP(B.SS_FEATURES, hidden, depth, seed)
    xt = torch.tensor(X, dtype=torch.float32, device=device).contiguous()
    yt = torch.tensor(y, dtype=torch.float32, device=device).contiguous()
    loss = m.train(xt, yt, iters, lr)
    return m, loss


def same_params(a, b):
    return (a.k or 1) == (b.k or 1) and a.N == b.N and a.l == b.l and a.split.top_l1 == b.split.top_l1 \
        and a.split.leaf_log2 == b.split.leaf_log2 and a.pad_rows == b.pad_rows and a.zeta_exp == b.zeta_exp


def policy_times(reqs, timings, model=None):
    """Per request: time of the default rule's candidate, of the model's choice
    (if a model is given) and of the exhaustive best, all from the timing table."""
    rows = []
    arr = B.requests_array(reqs)
    if model is not None:
        model.choose(arr)
    for i, (r, (cands, ms, best)) in enumerate(zip(reqs, timings)):
        d = B.ss_default_params(r.len_g, r.g_limbs, r.len_h, r.h_limbs)
        t_def = next(t for c, t in zip(cands, ms) if same_params(c, d))
        t_mlp = None
        if model is not None:
            t_mlp = next(t for c, t in zip(cands, ms) if same_params(c, arr[i].params))
        rows.append(dict(default=t_def, mlp=t_mlp, best=ms[best], k1=ms[0]))
    return rows
