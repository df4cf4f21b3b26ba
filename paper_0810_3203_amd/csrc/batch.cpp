// Batched Schoenhage-Strassen products (many independent products of uneven
// lengths, each with its own ring, length and split) executed together.
//
// Requests are grouped by ring size W (one kernel instantiation per W).  A
// group owns one cell array holding, per request, the transform of g and the
// transform of h.  Pass p of every request's TFT(g) and TFT(h) (Alg. 1) runs in
// a few leaf-kernel launches (one per work-group shape class), the pointwise
// products of all requests run in one launch over an item list, and pass p of
// every ITFT (Alg. 2) runs likewise: the launch count no longer grows with the
// number of requests.  The whole launch sequence can be captured once into a
// hipGraph and replayed.
// Requests whose workspace would exceed the caller's limit are split into
// consecutive chunks that reuse the same workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "../../include/tft.h"
#include "kernels.hpp"
#include "plan.hpp"
#include "ss.hpp"

using namespace tft;

namespace {

uint32_t fermat_max_leaf_log2(uint32_t W) {
    const uint64_t cap = lds_budget_bytes() / fermat_lds_cell_bytes(W);
    uint32_t lg = 0;
    while ((2ull << lg) <= cap) lg++;
    return std::min<uint32_t>(lg, 11);
}

// Leaf of a batch (unless a request asks for a smaller one): the largest whose
// cells fit a quarter of the LDS, so that four workgroups share a CU and one's
// copies overlap another's butterflies; at least 16 cells, so that large
// elements do not take many more passes.  (4096 requests of 256-limb cells:
// 128-cell leaves 1005 ms, 64: 1067 ms, 32: 866 ms, 16: 861 ms.)
uint32_t batch_leaf_log2(uint32_t W) {
    const uint64_t q = (lds_budget_bytes() / 4) / fermat_lds_cell_bytes(W);
    uint32_t lg = 0;
    while ((2ull << lg) <= q) lg++;
    return std::min(fermat_max_leaf_log2(W), std::max<uint32_t>(4, lg));
}

struct Pass {
    uint32_t job_begin, job_count, max_len, nwaves, opmask;
};

struct Group {
    uint32_t W = 0;
    uint64_t cap = 0;        // cells of the group's cell array
    uint64_t ws_offset = 0;  // byte offset of the cell array in the workspace
    std::vector<Job> jobs;
    std::vector<LeafProg> progs;
    std::vector<LeafStep> steps;
    std::vector<LeafOp> ops;
    std::vector<Pass> p1, p2;  // TFT passes, ITFT passes
    std::vector<uint4> items;
    std::vector<PackDesc> packs;
    std::vector<UnpackDesc> unpack1, unpackk;
    uint64_t max_z = 0, max_len1 = 0, max_lenk = 0;
    uint32_t max_ol1 = 0, max_olk = 0;
    // device copies
    void *dev = nullptr;
    Job *d_jobs = nullptr;
    LeafProg *d_progs = nullptr;
    LeafStep *d_steps = nullptr;
    LeafOp *d_ops = nullptr;
    uint4 *d_items = nullptr;
    PackDesc *d_packs = nullptr;
    UnpackDesc *d_unpack1 = nullptr, *d_unpackk = nullptr;
};

struct Chunk {
    std::vector<Group> groups;
    uint64_t bytes = 0;
};

// Adds a schedule's programs to the group's tables; returns the program offset.
uint32_t append_programs(Group &G, const Schedule &S) {
    const uint32_t prog0 = (uint32_t)G.progs.size(), step0 = (uint32_t)G.steps.size(), op0 = (uint32_t)G.ops.size();
    for (LeafProg p : S.progs) {
        p.step_begin += step0;
        G.progs.push_back(p);
    }
    for (LeafStep st : S.steps) {
        st.op_begin += op0;
        G.steps.push_back(st);
    }
    G.ops.insert(G.ops.end(), S.ops.begin(), S.ops.end());
    return prog0;
}

}  // namespace

struct tft_batch_plan {
    std::vector<Chunk> chunks;
    std::vector<int> status;
    std::vector<tft_ss_params> params;  // what each request was planned with
    uint64_t ws_bytes = 0;
    bool uploaded = false;
    int dev_id = -1;
    hipStream_t capture = nullptr;  // stream that graph captures record on
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *graph_ws = nullptr;
};

namespace {

int upload_group(Group &G) {
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t bj = al(G.jobs.size() * sizeof(Job)), bp = al(G.progs.size() * sizeof(LeafProg));
    const size_t bs = al(G.steps.size() * sizeof(LeafStep)), bo = al(G.ops.size() * sizeof(LeafOp));
    const size_t bi = al(G.items.size() * sizeof(uint4)), bk = al(G.packs.size() * sizeof(PackDesc));
    const size_t b1 = al(G.unpack1.size() * sizeof(UnpackDesc)), b2 = al(G.unpackk.size() * sizeof(UnpackDesc));
    const size_t total = bj + bp + bs + bo + bi + bk + b1 + b2 + 256;
    hipError_t me = hipMalloc(&G.dev, total);
    if (me != hipSuccess) return device_error(me, "batch: hipMalloc of descriptors");
    char *c = static_cast<char *>(G.dev);
    size_t off = 0;
    hipError_t e = hipSuccess;
    auto put = [&](const void *src, size_t n, size_t room) {
        void *dst = c + off;
        if (n && e == hipSuccess) e = hipMemcpy(dst, src, n, hipMemcpyHostToDevice);
        off += room;
        return dst;
    };
    G.d_jobs = static_cast<Job *>(put(G.jobs.data(), G.jobs.size() * sizeof(Job), bj));
    G.d_progs = static_cast<LeafProg *>(put(G.progs.data(), G.progs.size() * sizeof(LeafProg), bp));
    G.d_steps = static_cast<LeafStep *>(put(G.steps.data(), G.steps.size() * sizeof(LeafStep), bs));
    G.d_ops = static_cast<LeafOp *>(put(G.ops.data(), G.ops.size() * sizeof(LeafOp), bo));
    G.d_items = static_cast<uint4 *>(put(G.items.data(), G.items.size() * sizeof(uint4), bi));
    G.d_packs = static_cast<PackDesc *>(put(G.packs.data(), G.packs.size() * sizeof(PackDesc), bk));
    G.d_unpack1 = static_cast<UnpackDesc *>(put(G.unpack1.data(), G.unpack1.size() * sizeof(UnpackDesc), b1));
    G.d_unpackk = static_cast<UnpackDesc *>(put(G.unpackk.data(), G.unpackk.size() * sizeof(UnpackDesc), b2));
    return e == hipSuccess ? TFT_OK : device_error(e, "batch: descriptor upload");
}

hipError_t run_passes(const Group &G, const std::vector<Pass> &passes, uint32_t *x, hipStream_t st) {
    const uint32_t ord_mask = 64u * G.W - 1u;
    for (const Pass &p : passes) {
        hipError_t e = launch_fermat_leaf(G.W, p.nwaves, p.job_count, p.max_len, G.d_jobs, p.job_begin, G.d_progs,
                                          G.d_steps, G.d_ops, x, G.cap, ord_mask, p.opmask, true, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t run_plan(tft_batch_plan *P, char *ws, hipStream_t st) {
    const PackDesc np{};
    const UnpackDesc nu{};
    for (const Chunk &C : P->chunks) {
        for (const Group &G : C.groups) {
            uint32_t *x = reinterpret_cast<uint32_t *>(ws + G.ws_offset);
            hipError_t e =
                launch_fermat_pack(G.W, G.d_packs, (uint32_t)G.packs.size(), np, G.max_z, x, G.cap, true, st);
            if (e == hipSuccess) e = run_passes(G, G.p1, x, st);
            if (e == hipSuccess)
                e = launch_fermat_pointwise_items(G.W, G.items.size(), x, G.cap, G.d_items, true, st);
            if (e == hipSuccess) e = run_passes(G, G.p2, x, st);
            if (e == hipSuccess && !G.unpack1.empty())
                e = launch_fermat_unpack(G.W, G.d_unpack1, (uint32_t)G.unpack1.size(), nu, G.max_len1, G.max_ol1,
                                         false, x, G.cap, true, st);
            if (e == hipSuccess && !G.unpackk.empty())
                e = launch_fermat_unpack(G.W, G.d_unpackk, (uint32_t)G.unpackk.size(), nu, G.max_lenk, G.max_olk,
                                         true, x, G.cap, true, st);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// Uploads every group's descriptors and makes the capture stream on the
// current device.
int plan_prepare(tft_batch_plan *P) {
    int dev = 0;
    hipError_t ge = hipGetDevice(&dev);
    if (ge != hipSuccess) return device_error(ge, "batch: hipGetDevice");
    for (Chunk &C : P->chunks)
        for (Group &G : C.groups) {
            int rc = upload_group(G);
            if (rc) return rc;
        }
    hipError_t ce = hipStreamCreateWithFlags(&P->capture, hipStreamNonBlocking);
    if (ce != hipSuccess) {
        P->capture = nullptr;
        return device_error(ce, "batch: hipStreamCreateWithFlags");
    }
    P->uploaded = true;
    P->dev_id = dev;
    return TFT_OK;
}

}  // namespace

extern "C" {

int tft_batch_plan_create(const tft_zx_request *reqs_in, uint32_t count, uint64_t max_workspace, int policy,
                          tft_mlp *model, tft_batch_plan **plan) {
    if (!plan || (!reqs_in && count)) return TFT_E_ARG;
    if (policy != TFT_POLICY_GIVEN && policy != TFT_POLICY_RULE && policy != TFT_POLICY_MODEL) return TFT_E_ARG;
    if (policy == TFT_POLICY_MODEL && !model) return TFT_E_ARG;
    // the parameters every request is planned with
    std::vector<tft_zx_request> rq(reqs_in, reqs_in + count);
    if (policy == TFT_POLICY_RULE) {
        for (tft_zx_request &r : rq) {
            tft_ss_params d{};
            if (tft_ss_default_params(r.len_g, r.g_limbs, r.len_h, r.h_limbs, &d) == TFT_OK) r.params = d;
        }
    } else if (policy == TFT_POLICY_MODEL && count) {
        const int rc = tft_mlp_choose_ss(model, rq.data(), count, nullptr);
        if (rc) return rc;
    }
    const tft_zx_request *reqs = rq.data();
    tft_batch_plan *P = new tft_batch_plan();
    P->status.assign(count, TFT_OK);
    P->params.resize(count);
    for (uint32_t i = 0; i < count; i++) P->params[i] = rq[i].params;
    std::vector<SSShape> shapes(count);
    for (uint32_t i = 0; i < count; i++) {
        const tft_zx_request &r = reqs[i];
        int st = (!r.g || !r.h || !r.out) ? TFT_E_ARG
                                          : ss_shape(r.len_g, r.g_limbs, r.len_h, r.h_limbs, &r.params, &shapes[i]);
        if (!st && 32ull * r.out_limbs < shapes[i].bits) st = TFT_E_RANGE;
        if (!st && r.params.split.top_l1 && r.params.split.top_l1 != TFT_SPLIT_DC &&
            r.params.split.top_l1 >= shapes[i].l)
            st = TFT_E_ARG;
        if (!st && max_workspace && ((shapes[i].bytes + 255) & ~255ull) > max_workspace) st = TFT_E_WORKSPACE;
        P->status[i] = st;
    }
    // chunks of consecutive valid requests within the workspace limit
    std::vector<std::vector<uint32_t>> chunk_reqs;
    uint64_t cur = 0;
    for (uint32_t i = 0; i < count; i++) {
        if (P->status[i]) continue;
        const uint64_t b = (shapes[i].bytes + 255) & ~255ull;  // group arrays start at 256-byte boundaries
        if (chunk_reqs.empty() || (max_workspace && cur + b > max_workspace)) {
            chunk_reqs.emplace_back();
            cur = 0;
        }
        chunk_reqs.back().push_back(i);
        cur += b;
    }
    for (const auto &cr : chunk_reqs) {
        Chunk C;
        std::map<uint32_t, std::vector<uint32_t>> by_w;
        for (uint32_t i : cr) by_w[shapes[i].W].push_back(i);
        uint64_t byte_off = 0;
        for (const auto &kv : by_w) {
            Group G;
            G.W = kv.first;
            const uint32_t ord = 64u * G.W;
            std::map<std::tuple<uint32_t, uint32_t, uint32_t, uint64_t, uint64_t, uint32_t, uint32_t>,
                     std::pair<Schedule, uint32_t>>
                cache;
            auto sched = [&](uint32_t dir, uint32_t l, uint32_t s, uint64_t z, uint64_t n, uint32_t top,
                             uint32_t leaf) -> const std::pair<Schedule, uint32_t> & {
                auto key = std::make_tuple(dir, l, s, z, n, top, leaf);
                auto it = cache.find(key);
                if (it != cache.end()) return it->second;
                Schedule S = build_schedule(dir, l, ord, s, z, n, 0, leaf, top);
                const uint32_t off = append_programs(G, S);
                return cache.emplace(key, std::make_pair(std::move(S), off)).first->second;
            };
            std::vector<uint64_t> offA, offB;
            std::vector<const std::pair<Schedule, uint32_t> *> sg, sh, si;
            for (uint32_t i : kv.second) {
                const SSShape &s = shapes[i];
                const tft_zx_request &r = reqs[i];
                offA.push_back(G.cap);
                G.cap += s.L;
                offB.push_back(G.cap);
                G.cap += s.L;
                uint32_t leaf = batch_leaf_log2(G.W);
                if (r.params.split.leaf_log2)
                    leaf = std::min(fermat_max_leaf_log2(G.W), std::max<uint32_t>(1, r.params.split.leaf_log2));
                const uint32_t top = r.params.split.top_l1;
                sg.push_back(&sched(0, s.l, s.s, s.zg, s.nt, top, leaf));
                sh.push_back(&sched(0, s.l, s.s, s.zh, s.nt, top, leaf));
                si.push_back(&sched(1, s.l, (uint32_t)((2ull * s.s) % ord), s.nt, s.nt, top, leaf));
            }
            const uint32_t G64 = 64u / std::min<uint32_t>(G.W, 64u);
            // Pass p of every request runs in launches of its own, one per
            // class of work-group shape: the cells of the pass's longest job
            // (rounded up to a power of two) and the waves its largest step
            // needs.  One launch sizes LDS and waves for its largest job, so a
            // few long or wide programs in a launch would otherwise slow every
            // job beside them; a class of fewer than kMinClassJobs jobs joins
            // the next larger one instead of taking a launch of its own.
            auto merge = [&](std::vector<Pass> &out, const std::vector<std::vector<const std::pair<Schedule, uint32_t> *>> &lists,
                             const std::vector<std::vector<uint64_t>> &offs) {
                constexpr size_t kMinClassJobs = 512;
                struct Class {
                    std::vector<Job> jobs;
                    uint32_t max_len = 0, max_ops = 0, opmask = 0;
                };
                size_t np = 0;
                for (const auto &lst : lists)
                    for (const auto *s : lst) np = std::max(np, s->first.passes.size());
                for (size_t p = 0; p < np; p++) {
                    std::map<std::pair<uint32_t, uint32_t>, Class> classes;
                    for (size_t li = 0; li < lists.size(); li++) {
                        for (size_t q = 0; q < lists[li].size(); q++) {
                            const Schedule &S = lists[li][q]->first;
                            if (p >= S.passes.size()) continue;
                            const PassDesc &pd = S.passes[p];
                            if (!pd.job_count) continue;
                            uint32_t len2 = 1;
                            while (len2 < pd.max_len) len2 <<= 1;
                            const uint32_t waves = std::min<uint32_t>(8, std::max<uint32_t>(1, (pd.max_ops + G64 - 1) / G64));
                            Class &K = classes[{len2, waves}];
                            for (uint32_t j = 0; j < pd.job_count; j++) {
                                Job jb = S.jobs[pd.job_begin + j];
                                jb.base += offs[li][q];
                                jb.prog += lists[li][q]->second;
                                K.jobs.push_back(jb);
                            }
                            K.max_len = std::max(K.max_len, pd.max_len);
                            K.max_ops = std::max(K.max_ops, pd.max_ops);
                            K.opmask |= pd.opmask;
                        }
                    }
                    Class carry;
                    size_t left = classes.size();
                    for (auto &kc : classes) {
                        Class &K = kc.second;
                        carry.jobs.insert(carry.jobs.end(), K.jobs.begin(), K.jobs.end());
                        carry.max_len = std::max(carry.max_len, K.max_len);
                        carry.max_ops = std::max(carry.max_ops, K.max_ops);
                        carry.opmask |= K.opmask;
                        if (--left && carry.jobs.size() < kMinClassJobs) continue;
                        Pass ps{(uint32_t)G.jobs.size(), (uint32_t)carry.jobs.size(), carry.max_len, 1, carry.opmask};
                        ps.nwaves = std::min<uint32_t>(8, std::max<uint32_t>(1, (carry.max_ops + G64 - 1) / G64));
                        G.jobs.insert(G.jobs.end(), carry.jobs.begin(), carry.jobs.end());
                        if (ps.job_count) out.push_back(ps);
                        carry = Class{};
                    }
                }
            };
            merge(G.p1, {sg, sh}, {offA, offB});
            merge(G.p2, {si}, {offA});
            for (size_t q = 0; q < kv.second.size(); q++) {
                const uint32_t i = kv.second[q];
                const SSShape &s = shapes[i];
                const tft_zx_request &r = reqs[i];
                const uint32_t e = (uint32_t)((2ull * s.N - s.l) % (2ull * s.N));
                for (uint64_t c = 0; c < s.nt; c++)
                    G.items.push_back(make_uint4((uint32_t)(offA[q] + c), (uint32_t)(offB[q] + c), e, 0u));
                G.packs.push_back({r.g, r.len_g, offA[q], s.zg, r.g_limbs, s.k, s.ws, 0});
                G.packs.push_back({r.h, r.len_h, offB[q], s.zh, r.h_limbs, s.k, s.ws, 0});
                G.max_z = std::max(G.max_z, std::max(s.zg, s.zh));
                const uint64_t lo = r.len_g + r.len_h - 1;
                const UnpackDesc ud{r.out, lo, offA[q], s.n, r.out_limbs, s.k, s.ws, 0};
                if (s.k > 1) {
                    G.unpackk.push_back(ud);
                    G.max_lenk = std::max(G.max_lenk, lo);
                    G.max_olk = std::max(G.max_olk, r.out_limbs);
                } else {
                    G.unpack1.push_back(ud);
                    G.max_len1 = std::max(G.max_len1, lo);
                    G.max_ol1 = std::max(G.max_ol1, r.out_limbs);
                }
            }
            if (G.cap > 0xFFFFFFFFull) {
                delete P;
                return TFT_E_UNSUPPORTED;
            }
            G.ws_offset = byte_off;
            byte_off += (G.cap * (G.W + 1) * 4ull + 255) & ~255ull;
            C.groups.push_back(std::move(G));
        }
        C.bytes = byte_off;
        P->ws_bytes = std::max(P->ws_bytes, C.bytes);
        P->chunks.push_back(std::move(C));
    }
    // descriptors and the capture stream are made now, on the current device,
    // so that executions allocate nothing; without a device the plan stays
    // host-only (its workspace, status and launch counts can be read)
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
        int rc = plan_prepare(P);
        if (rc) {
            tft_batch_plan_destroy(P);
            return rc;
        }
    } else {
        (void)hipGetLastError();
    }
    *plan = P;
    return TFT_OK;
}

int tft_batch_plan_params(const tft_batch_plan *plan, tft_ss_params *params) {
    if (!plan || (!params && !plan->params.empty())) return TFT_E_ARG;
    std::copy(plan->params.begin(), plan->params.end(), params);
    return TFT_OK;
}

uint64_t tft_batch_plan_workspace(const tft_batch_plan *plan) { return plan ? plan->ws_bytes : 0; }

int tft_batch_plan_status(const tft_batch_plan *plan, int *status) {
    if (!plan || !status) return TFT_E_ARG;
    std::copy(plan->status.begin(), plan->status.end(), status);
    return TFT_OK;
}

uint32_t tft_batch_plan_launches(const tft_batch_plan *plan) {
    if (!plan) return 0;
    uint32_t n = 0;
    for (const Chunk &C : plan->chunks)
        for (const Group &G : C.groups)
            n += 2u + (uint32_t)G.p1.size() + (uint32_t)G.p2.size() + (G.unpack1.empty() ? 0u : 1u) +
                 (G.unpackk.empty() ? 0u : 1u);
    return n;
}

int tft_batch_plan_execute(tft_batch_plan *plan, void *ws, uint64_t ws_bytes, int use_graph, void *stream) {
    if (!plan || (!ws && plan->ws_bytes)) return TFT_E_ARG;
    if (ws_bytes < plan->ws_bytes) return TFT_E_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int dev = 0;
    hipError_t de = hipGetDevice(&dev);
    if (de != hipSuccess) return device_error(de, "batch: hipGetDevice");
    if (!plan->uploaded) {
        int rc = plan_prepare(plan);  // created without a device present
        if (rc) return rc;
    }
    if (dev != plan->dev_id) return TFT_E_ARG;  // descriptors live on the creating device
    char *w = static_cast<char *>(ws);
    if (!use_graph) {
        hipError_t e = run_plan(plan, w, st);
        return e == hipSuccess ? TFT_OK : device_error(e, "batch: launch");
    }
    if (!plan->exec || plan->graph_ws != ws) {
        // run once eagerly (sets kernel attributes outside capture), then capture
        hipError_t re = run_plan(plan, w, st);
        if (re != hipSuccess) return device_error(re, "batch: launch");
        if (plan->exec) {
            (void)hipGraphExecDestroy(plan->exec);
            (void)hipGraphDestroy(plan->graph);
            plan->exec = nullptr;
            plan->graph = nullptr;
        }
        hipStream_t cs = plan->capture;
        hipError_t e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = run_plan(plan, w, cs);
            e = hipStreamEndCapture(cs, &plan->graph);
            if (le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return device_error(e, "batch: graph capture");
        plan->graph_ws = ws;
        return TFT_OK;  // the eager run already produced this call's results
    }
    hipError_t ge = hipGraphLaunch(plan->exec, st);
    return ge == hipSuccess ? TFT_OK : device_error(ge, "batch: hipGraphLaunch");
}

void tft_batch_plan_destroy(tft_batch_plan *plan) {
    if (!plan) return;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->capture) (void)hipStreamDestroy(plan->capture);
    for (Chunk &C : plan->chunks)
        for (Group &G : C.groups)
            if (G.dev) (void)hipFree(G.dev);
    delete plan;
}

}  // extern "C"
