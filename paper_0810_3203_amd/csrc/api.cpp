// C ABI of the library (include/tft.h): argument checks, plan cache, and the
// sequencing of kernels for the transforms and the two products.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/tft.h"
#include "kernels.hpp"
#include "nega.hpp"
#include "plan.hpp"
#include "prime.hpp"
#include "ss.hpp"

static_assert(tft::kSplitDC == TFT_SPLIT_DC, "divide-and-conquer split code");

using namespace tft;

struct tft_plan {
    tft_ring ring;
    uint32_t direction, l;
    uint64_t s, z, n;
    uint32_t f;
    Schedule sched;
    std::vector<uint32_t> nwaves;  // per pass
    void *dev = nullptr;           // device copy of the descriptor blob (plan-owned)
    int dev_id = -1;
    std::vector<char> blob;        // jobs | progs | steps | ops, 256-byte aligned tables
    size_t bj = 0, bp = 0, bs = 0, bo = 0;
    Job *d_jobs = nullptr;
    LeafProg *d_progs = nullptr;
    LeafStep *d_steps = nullptr;
    LeafOp *d_ops = nullptr;
    // Z/pZ only: per-op twiddles (Montgomery theta^b; theta^-b for the inverse
    // butterfly) and the twist-table width (every op's alog < zw)
    std::vector<uint32_t> optw;
    uint32_t zw = 0;
    size_t bw = 0;
    uint32_t *d_optw = nullptr;
    std::mutex mu;
};

namespace {

bool is_pow2(uint64_t v) { return v && !(v & (v - 1)); }

uint32_t log2u(uint64_t v) {
    uint32_t l = 0;
    while ((1ull << l) < v) l++;
    return l;
}

int check_ring(const tft_ring *r) {
    if (!r) return TFT_E_ARG;
    if (r->kind == TFT_RING_FERMAT) {
        if (r->N == 0 || r->N % 32 || r->K || r->m) return TFT_E_RING;
        uint32_t W = r->N / 32;
        if (!is_pow2(W) || W > 4096) return TFT_E_RING;
        return TFT_OK;
    }
    if (r->kind == TFT_RING_NEGA) {
        if (r->N || !is_pow2(r->K) || r->K < 2 || r->K > 4096) return TFT_E_RING;
        if (r->m < 3 || !(r->m & 1) || r->m >= (1ull << 62)) return TFT_E_RING;
        return TFT_OK;
    }
    if (r->kind == TFT_RING_PRIME) {
        if (r->N || r->K || r->reserved || r->m != zp::P) return TFT_E_RING;
        return TFT_OK;
    }
    return TFT_E_RING;
}

uint32_t ring_ord(const tft_ring *r) {
    if (r->kind == TFT_RING_PRIME) return zp::ORD;
    return r->kind == TFT_RING_FERMAT ? 2u * r->N : 2u * r->K;
}

// LDS bytes of one cell inside a leaf workgroup
uint64_t cell_lds_bytes(const tft_ring *r) {
    if (r->kind == TFT_RING_PRIME) return 4;
    return r->kind == TFT_RING_FERMAT ? fermat_lds_cell_bytes(r->N / 32) : 8ull * r->K;
}

uint32_t max_leaf_log2(const tft_ring *r) {
    // Z/pZ: leaves of 2^12 words (16 KB), so that with balanced splits a
    // transform of up to 2^24 cells takes two passes
    if (r->kind == TFT_RING_PRIME) return 12;
    uint64_t cap = lds_budget_bytes() / cell_lds_bytes(r);
    uint32_t lg = 0;
    while ((2ull << lg) <= cap) lg++;
    return std::min<uint32_t>(lg, 11);
}

// log2 of twice the compute units of the current device (cached per device)
uint32_t fill_log2() {
    static uint32_t cache[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 9;
    if (!cache[dev]) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
        uint32_t lg = 0;
        while ((1u << lg) < 2u * (uint32_t)cus) lg++;
        cache[dev] = lg;
    }
    return cache[dev];
}

thread_local char g_last_error[256] = "";

// Records the HIP error of a failed call (readable through tft_last_error) and
// prints it when TFT_DEBUG is set in the environment.
int dev_fail(hipError_t e, const char *where) {
    snprintf(g_last_error, sizeof g_last_error, "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
    if (getenv("TFT_DEBUG")) fprintf(stderr, "[tft] %s\n", g_last_error);
    return TFT_E_DEVICE;
}

int hip_status(hipError_t e, const char *where = "launch") { return e == hipSuccess ? TFT_OK : dev_fail(e, where); }

int check_transform_args(const tft_ring *ring, uint32_t dir, uint32_t l, uint64_t z, uint64_t n, uint32_t f) {
    int st = check_ring(ring);
    if (st) return st;
    if (l < 1 || l > (ring->kind == TFT_RING_PRIME ? zp::ORD_LOG2 : 24u)) return TFT_E_ARG;
    const uint64_t L = 1ull << l;
    if (ring_ord(ring) % L) return TFT_E_RING;
    if (dir == 0) {
        if (z < 1 || z > L || n < 1 || n > L) return TFT_E_ARG;
    } else {
        if (f > 1 || z < 1 || z > L || z < n || n + f < 1 || n + f > L) return TFT_E_ARG;
    }
    return TFT_OK;
}

// The plan's descriptors as one host blob: jobs | programs | steps | ops,
// each table 256-byte aligned.  Built once per plan; copied to the device at
// tft_plan_create (plan-owned memory) or, for the one-call transforms, into
// the caller's workspace on every call.
void plan_blob(tft_plan *p) {
    if (!p->blob.empty()) return;
    const Schedule &S = p->sched;
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    p->bj = al(S.jobs.size() * sizeof(Job));
    p->bp = al(S.progs.size() * sizeof(LeafProg));
    p->bs = al(S.steps.size() * sizeof(LeafStep));
    p->bo = al(std::max<size_t>(1, S.ops.size()) * sizeof(LeafOp));
    p->bw = p->optw.empty() ? 0 : al(p->optw.size() * sizeof(uint32_t));
    p->blob.assign(p->bj + p->bp + p->bs + p->bo + p->bw, 0);
    char *c = p->blob.data();
    if (!S.jobs.empty()) memcpy(c, S.jobs.data(), S.jobs.size() * sizeof(Job));
    if (!S.progs.empty()) memcpy(c + p->bj, S.progs.data(), S.progs.size() * sizeof(LeafProg));
    if (!S.steps.empty()) memcpy(c + p->bj + p->bp, S.steps.data(), S.steps.size() * sizeof(LeafStep));
    if (!S.ops.empty()) memcpy(c + p->bj + p->bp + p->bs, S.ops.data(), S.ops.size() * sizeof(LeafOp));
    if (p->bw) memcpy(c + p->bj + p->bp + p->bs + p->bo, p->optw.data(), p->optw.size() * sizeof(uint32_t));
}

// Descriptor pointers of a blob placed at device address d.
void plan_point(tft_plan *p, void *d) {
    char *c = static_cast<char *>(d);
    p->d_jobs = reinterpret_cast<Job *>(c);
    p->d_progs = reinterpret_cast<LeafProg *>(c + p->bj);
    p->d_steps = reinterpret_cast<LeafStep *>(c + p->bj + p->bp);
    p->d_ops = reinterpret_cast<LeafOp *>(c + p->bj + p->bp + p->bs);
    p->d_optw = p->bw ? reinterpret_cast<uint32_t *>(c + p->bj + p->bp + p->bs + p->bo) : nullptr;
}

int plan_upload(tft_plan *p) {
    int dev = 0;
    hipError_t ge = hipGetDevice(&dev);
    if (ge != hipSuccess) return dev_fail(ge, "hipGetDevice");
    if (p->dev && p->dev_id == dev) {
        plan_point(p, p->dev);
        return TFT_OK;
    }
    plan_blob(p);
    void *buf = nullptr;
    hipError_t me = hipMalloc(&buf, p->blob.size());
    if (me != hipSuccess) return dev_fail(me, "hipMalloc(plan)");
    hipError_t e = hipMemcpy(buf, p->blob.data(), p->blob.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(buf);
        return dev_fail(e, "hipMemcpy(plan)");
    }
    if (p->dev) (void)hipFree(p->dev);
    p->dev = buf;
    p->dev_id = dev;
    plan_point(p, p->dev);
    return TFT_OK;
}

// Z/pZ plans: each pass's jobs in order of (stride, first cell), so that a
// workgroup's pack of jobs is adjacent columns (or rows); the per-op twiddle
// table; the twist-table width.  Jobs of a pass are independent, their order
// changes no output.
void zp_prepare(tft_plan *p) {
    Schedule &S = p->sched;
    for (const PassDesc &pd : S.passes)
        std::stable_sort(S.jobs.begin() + pd.job_begin, S.jobs.begin() + pd.job_begin + pd.job_count,
                         [](const Job &a, const Job &b) {
                             return a.stride != b.stride ? a.stride < b.stride : a.base < b.base;
                         });
    p->optw.resize(S.ops.size());
    uint32_t amax = 0;
    for (size_t i = 0; i < S.ops.size(); i++) {
        const LeafOp &o = S.ops[i];
        const uint32_t b = op_b(o);
        amax = std::max(amax, op_alog(o));
        const uint64_t e = (o.w0 & 15u) == OP_I2 ? (uint64_t)zp::ORD - b : b;
        p->optw[i] = zp::theta_pow_m(e);
    }
    p->zw = amax + 1u;
    // the kernel loads a step's ops while the previous step runs, taking them
    // to follow that step's ops directly; a plan that breaks this is refused
    // at launch (zw = 0)
    for (const LeafProg &P : S.progs)
        for (uint32_t st = 1; st < P.step_count; st++) {
            const LeafStep &a = S.steps[P.step_begin + st - 1], &b = S.steps[P.step_begin + st];
            if (b.op_begin != a.op_begin + a.op_count) p->zw = 0;
        }
}

tft_plan *plan_build(const tft_ring *ring, uint32_t dir, uint32_t l, uint64_t s, uint64_t z, uint64_t n, uint32_t f,
                     const tft_split *split) {
    tft_plan *p = new tft_plan();
    p->ring = *ring;
    p->direction = dir;
    p->l = l;
    p->s = s % ring_ord(ring);
    p->z = z;
    p->n = n;
    p->f = dir ? f : 0;
    // an explicit leaf size is honoured as given (a plan is host data); plans whose
    // leaves exceed the LDS budget are refused when executed
    const bool prime = ring->kind == TFT_RING_PRIME;
    uint32_t leaf = max_leaf_log2(ring);
    if (split && split->leaf_log2) leaf = std::min<uint32_t>(prime ? 12 : 11, split->leaf_log2);
    uint32_t top = 0;
    if (split && split->top_l1 && (split->top_l1 == kSplitDC || split->top_l1 < l)) top = split->top_l1;
    p->sched = build_schedule(dir, l, ring_ord(ring), p->s, z, n, p->f, leaf, top, prime);
    if (prime) zp_prepare(p);
    const uint32_t seg = ring->kind == TFT_RING_FERMAT ? std::min<uint32_t>(ring->N / 32, 64) : 64;
    const uint32_t G = 64 / seg;
    for (const PassDesc &pd : p->sched.passes) {
        uint32_t w = (pd.max_ops + G - 1) / G;
        p->nwaves.push_back(std::min<uint32_t>(8, std::max<uint32_t>(1, w)));
    }
    return p;
}

// Optional per-launch event pairs, for timing the leaf kernels on their stream.
// Event pairs are created up front (reserve) so that timing adds only the
// event records between launches.
struct LaunchTimer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
    ~LaunchTimer() {
        for (auto &e : ev) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    }
    hipError_t reserve(size_t n) {
        while (ev.size() < n) {
            std::pair<hipEvent_t, hipEvent_t> p;
            hipError_t e = hipEventCreate(&p.first);
            if (e != hipSuccess) return e;
            e = hipEventCreate(&p.second);
            if (e != hipSuccess) {
                (void)hipEventDestroy(p.first);
                return e;
            }
            ev.push_back(p);
        }
        return hipSuccess;
    }
    hipError_t mark(hipStream_t st, bool start) {
        if (start) {
            if (used == ev.size()) {
                hipError_t e = reserve(used + 1);
                if (e != hipSuccess) return e;
            }
            return hipEventRecord(ev[used++].first, st);
        }
        return hipEventRecord(ev[used - 1].second, st);
    }
    float total_ms() {
        float t = 0;
        for (size_t i = 0; i < used; i++) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, ev[i].first, ev[i].second) == hipSuccess) t += ms;
        }
        return t;
    }
};

bool plan_fits(const tft_plan *p) {
    for (const PassDesc &pd : p->sched.passes)
        if ((uint64_t)pd.max_len * cell_lds_bytes(&p->ring) > lds_budget_bytes()) return false;
    return true;
}

// Launches the passes with the descriptor pointers already set (p->mu held).
int plan_launch(tft_plan *p, void *x, hipStream_t st, LaunchTimer *lt, bool transposed) {
    const uint64_t cap = 1ull << p->l;
    const uint32_t ord_mask = ring_ord(&p->ring) - 1;
    for (size_t i = 0; i < p->sched.passes.size(); i++) {
        const PassDesc &pd = p->sched.passes[i];
        hipError_t e = hipSuccess;
        if (lt && (e = lt->mark(st, true)) != hipSuccess) return dev_fail(e, "timer");
        if (p->ring.kind == TFT_RING_PRIME)
            e = launch_zp_leaf(pd.job_count, pd.max_len, pd.max_ops, p->d_jobs, pd.job_begin, p->d_progs, p->d_steps, p->d_ops,
                               p->d_optw, static_cast<uint32_t *>(x), p->zw, st);
        else if (p->ring.kind == TFT_RING_FERMAT)
            e = launch_fermat_leaf(p->ring.N / 32, p->nwaves[i], pd.job_count, pd.max_len, p->d_jobs, pd.job_begin,
                                   p->d_progs, p->d_steps, p->d_ops, static_cast<uint32_t *>(x), cap, ord_mask,
                                   pd.opmask, transposed, st);
        else
            e = launch_nega_leaf(p->ring.K, p->ring.m, p->nwaves[i], pd.job_count, pd.max_len, p->d_jobs,
                                 pd.job_begin, p->d_progs, p->d_steps, p->d_ops, static_cast<uint64_t *>(x), ord_mask,
                                 st);
        if (e != hipSuccess) return dev_fail(e, "leaf pass");
        if (lt && (e = lt->mark(st, false)) != hipSuccess) return dev_fail(e, "timer");
    }
    return TFT_OK;
}

// Runs a plan from its plan-owned device descriptors (uploaded on first use).
int plan_run(tft_plan *p, void *x, hipStream_t st, LaunchTimer *lt = nullptr, bool transposed = false) {
    std::lock_guard<std::mutex> lk(p->mu);
    if (!plan_fits(p)) return TFT_E_UNSUPPORTED;
    int rc = plan_upload(p);
    if (rc) return rc;
    return plan_launch(p, x, st, lt, transposed);
}

// Runs a plan from descriptors copied into the caller's workspace on the
// stream (no device memory of the library's own).
int plan_run_ws(tft_plan *p, void *x, void *ws, uint64_t ws_bytes, hipStream_t st, LaunchTimer *lt = nullptr,
                bool transposed = false) {
    std::lock_guard<std::mutex> lk(p->mu);
    if (!plan_fits(p)) return TFT_E_UNSUPPORTED;
    plan_blob(p);
    if (!ws || ws_bytes < p->blob.size() || (reinterpret_cast<uintptr_t>(ws) & 255u)) return TFT_E_WORKSPACE;
    hipError_t e = hipMemcpyAsync(ws, p->blob.data(), p->blob.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return dev_fail(e, "hipMemcpyAsync(descriptors)");
    plan_point(p, ws);
    const int rc = plan_launch(p, x, st, lt, transposed);
    if (p->dev) plan_point(p, p->dev);
    return rc;
}

// cache of plans used by the one-call entry points
std::mutex g_cache_mu;
std::map<std::vector<uint64_t>, tft_plan *> g_cache;

tft_plan *cached_plan(const tft_ring *ring, uint32_t dir, uint32_t l, uint64_t s, uint64_t z, uint64_t n, uint32_t f,
                      const tft_split *split) {
    std::vector<uint64_t> key{ring->kind, ring->N, ring->K, ring->m, dir, l, s % ring_ord(ring), z, n, dir ? f : 0,
                              split ? split->top_l1 : 0, split ? split->leaf_log2 : 0};
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) return it->second;
    tft_plan *p = plan_build(ring, dir, l, s, z, n, f, split);
    g_cache[key] = p;
    return p;
}

}  // namespace

namespace tft {
int device_error(hipError_t e, const char *where) { return dev_fail(e, where); }

uint32_t ss_leaf_log2(uint32_t N, uint32_t l) {
    const tft_ring ring{TFT_RING_FERMAT, N, 0, 0, 0};
    const uint32_t fit = max_leaf_log2(&ring), fill = fill_log2();
    return (l > fill + 3) ? std::min(fit, std::max<uint32_t>(3, l - fill))
                          : std::min(fit, std::max<uint32_t>(1, (l + 1) / 2));
}
}  // namespace tft

extern "C" {

const char *tft_last_error(void) { return g_last_error; }

const char *tft_status_string(int status) {
    switch (status) {
        case TFT_OK: return "ok";
        case TFT_E_ARG: return "invalid argument";
        case TFT_E_RING: return "unsupported ring or no root of the needed order";
        case TFT_E_RANGE: return "output does not fit";
        case TFT_E_WORKSPACE: return "workspace missing or too small";
        case TFT_E_DEVICE: return "HIP device error";
        case TFT_E_UNSUPPORTED: return "not supported by this build";
        default: return "unknown status";
    }
}

int tft_ring_check(const tft_ring *ring) { return check_ring(ring); }

uint64_t tft_elem_bytes(const tft_ring *ring) {
    if (check_ring(ring)) return 0;
    if (ring->kind == TFT_RING_PRIME) return 4;
    return ring->kind == TFT_RING_FERMAT ? 4ull * (ring->N / 32 + 1) : 8ull * ring->K;
}

uint64_t tft_array_bytes(const tft_ring *ring, uint64_t cells) { return tft_elem_bytes(ring) * cells; }

int tft_plan_create(const tft_ring *ring, uint32_t direction, uint32_t l, uint64_t s, uint64_t z, uint64_t n,
                    uint32_t f, const tft_split *split, tft_plan **plan) {
    if (!plan || direction > 1) return TFT_E_ARG;
    int st = check_transform_args(ring, direction, l, z, n, f);
    if (st) return st;
    if (split && split->top_l1 && split->top_l1 != TFT_SPLIT_DC && split->top_l1 >= l) return TFT_E_ARG;
    tft_plan *p = plan_build(ring, direction, l, s, z, n, f, split);
    // descriptors go to the current device now, so that executing the plan
    // there allocates nothing.  Without a device (schedule inspection on a
    // host) and for leaves beyond the LDS the plan stays host-only.
    int ndev = 0;
    const bool have_dev = hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0;
    if (!have_dev) (void)hipGetLastError();
    if (have_dev && plan_fits(p)) {
        int rc = plan_upload(p);
        if (rc) {
            delete p;
            return rc;
        }
    }
    *plan = p;
    return TFT_OK;
}

int tft_plan_execute(tft_plan *plan, void *x, void *stream) {
    if (!plan || !x) return TFT_E_ARG;
    return plan_run(plan, x, static_cast<hipStream_t>(stream));
}

void tft_plan_destroy(tft_plan *plan) {
    if (!plan) return;
    if (plan->dev) (void)hipFree(plan->dev);
    delete plan;
}

uint64_t tft_plan_base_cases(const tft_plan *plan) { return plan ? plan->sched.base_cases : 0; }

int tft_plan_export(const tft_plan *plan, uint64_t *buf, uint64_t cap_words, uint64_t *needed) {
    if (!plan || !needed) return TFT_E_ARG;
    const Schedule &S = plan->sched;
    uint64_t words = 8 + 3 * S.passes.size() + 6 * S.jobs.size() + 3 * S.progs.size() + 2 * S.steps.size() +
                     5 * S.ops.size();
    *needed = words;
    if (!buf || cap_words < words) return TFT_E_ARG;
    uint64_t *w = buf;
    *w++ = 1;
    *w++ = S.passes.size();
    *w++ = S.jobs.size();
    *w++ = S.progs.size();
    *w++ = S.steps.size();
    *w++ = S.ops.size();
    *w++ = S.ord;
    *w++ = S.leaf_log2;
    for (const PassDesc &p : S.passes) {
        *w++ = p.job_begin;
        *w++ = p.job_count;
        *w++ = p.max_len;
    }
    for (const Job &j : S.jobs) {
        *w++ = j.base;
        *w++ = j.stride;
        *w++ = j.prog;
        *w++ = j.s;
        *w++ = j.nload;
        *w++ = j.nstore;
    }
    for (const LeafProg &p : S.progs) {
        *w++ = p.step_begin;
        *w++ = p.step_count;
        *w++ = p.len;
    }
    for (const LeafStep &s : S.steps) {
        *w++ = s.op_begin;
        *w++ = s.op_count;
    }
    for (const LeafOp &o : S.ops) {
        *w++ = o.w0 & 15u;
        *w++ = (o.w0 >> 4) & 16383u;
        *w++ = (o.w0 >> 18) & 16383u;
        *w++ = op_alog(o);
        *w++ = op_b(o);
    }
    return TFT_OK;
}

int tft_transform_workspace(const tft_ring *ring, uint32_t direction, uint32_t l, uint64_t s, uint64_t z, uint64_t n,
                            uint32_t f, uint64_t *bytes) {
    if (!bytes || direction > 1) return TFT_E_ARG;
    int st = check_transform_args(ring, direction, l, z, n, f);
    if (st) return st;
    tft_plan *p = cached_plan(ring, direction, l, s, z, n, f, nullptr);
    std::lock_guard<std::mutex> lk(p->mu);
    plan_blob(p);
    *bytes = p->blob.size();
    return TFT_OK;
}

int tft_forward(const tft_ring *ring, uint32_t l, uint64_t s, uint64_t z, uint64_t n, void *x, void *ws,
                uint64_t ws_bytes, void *stream) {
    int st = check_transform_args(ring, 0, l, z, n, 0);
    if (st) return st;
    if (!x) return TFT_E_ARG;
    return plan_run_ws(cached_plan(ring, 0, l, s, z, n, 0, nullptr), x, ws, ws_bytes,
                       static_cast<hipStream_t>(stream));
}

int itft_inverse(const tft_ring *ring, uint32_t l, uint64_t s, uint64_t z, uint64_t n, uint32_t f, void *x, void *ws,
                 uint64_t ws_bytes, void *stream) {
    int st = check_transform_args(ring, 1, l, z, n, f);
    if (st) return st;
    if (!x) return TFT_E_ARG;
    return plan_run_ws(cached_plan(ring, 1, l, s, z, n, f, nullptr), x, ws, ws_bytes,
                       static_cast<hipStream_t>(stream));
}

int tft_debug_base_cases(const tft_ring *ring, uint32_t ncases, const void *cases, void *out, void *stream) {
    int st = check_ring(ring);
    if (st) return st;
    if (ring->kind != TFT_RING_FERMAT || ring->N < 8192 || ring->N > 65536) return TFT_E_UNSUPPORTED;
    if (!cases || !out) return TFT_E_ARG;
    return hip_status(launch_base_case_probe(ring->N / 32, ncases, static_cast<const uint32_t *>(cases),
                                             static_cast<uint32_t *>(out), static_cast<hipStream_t>(stream)),
                      "base case probe");
}

int pointwise_mul(const tft_ring *ring, uint64_t n, const void *a, const void *b, void *c, uint64_t cap,
                  uint32_t scale_log2, void *stream) {
    int st = check_ring(ring);
    if (st) return st;
    if (!a || !b || !c || n > cap || n > 0xFFFFFFFFull) return TFT_E_ARG;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const uint32_t ord = ring_ord(ring);
    if (ring->kind == TFT_RING_PRIME)
        return hip_status(launch_zp_pointwise(n, static_cast<const uint32_t *>(a), static_cast<const uint32_t *>(b),
                                              static_cast<uint32_t *>(c), scale_log2, hs));
    if (ring->kind == TFT_RING_FERMAT) {
        const uint32_t e = (uint32_t)((ord - (scale_log2 % ord)) % ord);
        return hip_status(launch_fermat_pointwise(ring->N / 32, n, static_cast<const uint32_t *>(a),
                                                  static_cast<const uint32_t *>(b), static_cast<uint32_t *>(c), cap,
                                                  e, false, hs));
    }
    return hip_status(launch_nega_pointwise(ring->K, ring->m, n, static_cast<const uint64_t *>(a),
                                            static_cast<const uint64_t *>(b), static_cast<uint64_t *>(c),
                                            scale_log2, hs));
}

// ---------------------------------------------------------------------------
// Schoenhage-Strassen in Z[x] (Sect. 5.1)
// ---------------------------------------------------------------------------

int zx_mul_ss_workspace(uint64_t len_g, uint32_t g_limbs, uint64_t len_h, uint32_t h_limbs,
                        const tft_ss_params *params, uint64_t *bytes) {
    if (!bytes) return TFT_E_ARG;
    SSShape sh;
    int st = ss_shape(len_g, g_limbs, len_h, h_limbs, params, &sh);
    if (st) return st;
    *bytes = sh.bytes;
    return TFT_OK;
}

// The three transform plans of a product (TFT of g, TFT of h, ITFT).
struct SSPlans {
    SSShape sh;
    tft_plan *pg, *ph, *pi;
};

static int ss_plans(uint64_t len_g, uint32_t g_limbs, uint64_t len_h, uint32_t h_limbs, uint32_t out_limbs,
             const tft_ss_params *params, SSPlans *o) {
    SSShape &sh = o->sh;
    int st = ss_shape(len_g, g_limbs, len_h, h_limbs, params, &sh);
    if (st) return st;
    if (32ull * out_limbs < sh.bits) return TFT_E_RANGE;
    tft_ring ring{TFT_RING_FERMAT, sh.N, 0, 0, 0};
    // One product on its own: unless the caller chose the leaf, cap it so that a
    // pass still has about two leaf jobs per compute unit (larger leaves mean
    // fewer passes, but a pass of fewer jobs than CUs leaves the GPU part idle);
    // a small transform takes two passes of half its length rather than one
    // workgroup running every level alone.
    tft_split sp = params ? params->split : tft_split{0, 0};
    if (!sp.leaf_log2) sp.leaf_log2 = ss_leaf_log2(sh.N, sh.l);
    o->pg = cached_plan(&ring, 0, sh.l, sh.s, sh.zg, sh.nt, 0, &sp);
    o->ph = cached_plan(&ring, 0, sh.l, sh.s, sh.zh, sh.nt, 0, &sp);
    o->pi = cached_plan(&ring, 1, sh.l, (2ull * sh.s) % (2ull * sh.N), sh.nt, sh.nt, 0, &sp);
    return TFT_OK;
}

static uint64_t blob_bytes(tft_plan *p) {
    std::lock_guard<std::mutex> lk(p->mu);
    plan_blob(p);
    return p->blob.size();
}

// desc == nullptr: the plans run from their own device descriptors (uploaded
// on first use).  Otherwise the three plans' descriptors are copied into
// desc (desc_bytes >= the sum of their blobs) on the stream.
static int ss_run(const uint32_t *g, uint64_t len_g, uint32_t g_limbs, const uint32_t *h, uint64_t len_h, uint32_t h_limbs,
           uint32_t *out, uint32_t out_limbs, const tft_ss_params *params, void *ws, uint64_t ws_bytes,
           hipStream_t hs, tft_ss_timing *tm, char *desc = nullptr, uint64_t desc_bytes = 0) {
    if (!g || !h || !out) return TFT_E_ARG;
    SSPlans P;
    int st = ss_plans(len_g, g_limbs, len_h, h_limbs, out_limbs, params, &P);
    if (st) return st;
    const SSShape &sh = P.sh;
    if (!ws || ws_bytes < sh.bytes) return TFT_E_WORKSPACE;
    uint32_t *A = static_cast<uint32_t *>(ws);
    uint32_t *B = A + sh.L * (sh.W + 1);
    tft_plan *pg = P.pg, *ph = P.ph, *pi = P.pi;
    char *dg_at = nullptr, *dh_at = nullptr, *di_at = nullptr;
    uint64_t bg = 0, bh = 0, bi = 0;
    if (desc) {
        bg = blob_bytes(pg);
        bh = blob_bytes(ph);
        bi = blob_bytes(pi);
        if (desc_bytes < bg + bh + bi) return TFT_E_WORKSPACE;
        dg_at = desc;
        dh_at = desc + bg;
        di_at = desc + bg + bh;
    }
    hipEvent_t ev[7] = {};
    LaunchTimer lt;
    LaunchTimer *ltp = tm ? &lt : nullptr;
    if (tm) {
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) return dev_fail(hipErrorUnknown, "hipEventCreate");
        hipError_t re = lt.reserve(pg->sched.passes.size() + ph->sched.passes.size() + pi->sched.passes.size());
        if (re != hipSuccess) return dev_fail(re, "hipEventCreate");
    }
    auto mark = [&](int i) { return tm ? hipEventRecord(ev[i], hs) : hipSuccess; };
    hipError_t e = mark(0);
    const PackDesc dg{g, len_g, 0, sh.zg, g_limbs, sh.k, sh.ws, 0};
    const PackDesc dh{h, len_h, 0, sh.zh, h_limbs, sh.k, sh.ws, 0};
    if (e == hipSuccess) e = launch_fermat_pack(sh.W, nullptr, 1, dg, sh.zg, A, sh.L, true, hs);
    if (e == hipSuccess) e = launch_fermat_pack(sh.W, nullptr, 1, dh, sh.zh, B, sh.L, true, hs);
    if (e == hipSuccess) e = mark(1);
    if (e != hipSuccess) st = dev_fail(e, "pack");
    auto run = [&](tft_plan *p, uint32_t *x, char *d, uint64_t b) {
        return d ? plan_run_ws(p, x, d, b, hs, ltp, true) : plan_run(p, x, hs, ltp, true);
    };
    if (!st) st = run(pg, A, dg_at, bg);
    if (!st && (e = mark(2)) != hipSuccess) st = dev_fail(e, "event");
    if (!st) st = run(ph, B, dh_at, bh);
    if (!st && (e = mark(3)) != hipSuccess) st = dev_fail(e, "event");
    if (!st) {
        e = launch_fermat_pointwise(sh.W, sh.nt, A, B, A, sh.L, (uint32_t)((2 * sh.N - sh.l) % (2 * sh.N)), true, hs);
        if (e == hipSuccess) e = mark(4);
        if (e != hipSuccess) st = dev_fail(e, "pointwise");
    }
    if (!st) st = run(pi, A, di_at, bi);
    if (!st && (e = mark(5)) != hipSuccess) st = dev_fail(e, "event");
    if (!st) {
        const UnpackDesc du{out, len_g + len_h - 1, 0, sh.n, out_limbs, sh.k, sh.ws, 0};
        e = launch_fermat_unpack(sh.W, nullptr, 1, du, len_g + len_h - 1, out_limbs, sh.k > 1, A, sh.L, true, hs);
        if (e == hipSuccess) e = mark(6);
        if (e != hipSuccess) st = dev_fail(e, "unpack");
    }
    if (tm) {
        if (!st) {
            e = hipEventSynchronize(ev[6]);
            if (e != hipSuccess) st = dev_fail(e, "hipEventSynchronize");
        }
        if (!st) {
            float ms[6];
            for (int i = 0; i < 6; i++) (void)hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]);
            tm->pack_ms = ms[0];
            tm->tft_g_ms = ms[1];
            tm->tft_h_ms = ms[2];
            tm->pointwise_ms = ms[3];
            tm->itft_ms = ms[4];
            tm->unpack_ms = ms[5];
            (void)hipEventElapsedTime(&tm->total_ms, ev[0], ev[6]);
            tm->leaf_kernel_ms = lt.total_ms();
            tm->leaf_launches = (uint32_t)lt.used;
            tm->n = sh.n;
            tm->l = sh.l;
            tm->N = sh.N;
        }
        for (auto &x : ev) (void)hipEventDestroy(x);
    }
    return st;
}

}  // extern "C"

namespace tft {

// Bytes of one scratch area holding a product's cell arrays followed by its
// three plans' descriptors; 0 with *status set when the request is invalid.
int ss_scratch_bytes(uint64_t len_g, uint32_t g_limbs, uint64_t len_h, uint32_t h_limbs, uint32_t out_limbs,
                     const tft_ss_params *params, uint64_t *bytes) {
    SSPlans P;
    int st = ss_plans(len_g, g_limbs, len_h, h_limbs, out_limbs, params, &P);
    if (st) return st;
    *bytes = ((P.sh.bytes + 255) & ~255ull) + blob_bytes(P.pg) + blob_bytes(P.ph) + blob_bytes(P.pi);
    return TFT_OK;
}

int ss_scratch_run(const uint32_t *g, uint64_t len_g, uint32_t g_limbs, const uint32_t *h, uint64_t len_h,
                   uint32_t h_limbs, uint32_t *out, uint32_t out_limbs, const tft_ss_params *params, void *scratch,
                   uint64_t scratch_bytes, hipStream_t hs) {
    SSShape sh;
    int st = ss_shape(len_g, g_limbs, len_h, h_limbs, params, &sh);
    if (st) return st;
    const uint64_t cells = (sh.bytes + 255) & ~255ull;
    if (cells > scratch_bytes) return TFT_E_WORKSPACE;
    char *c = static_cast<char *>(scratch);
    return ss_run(g, len_g, g_limbs, h, len_h, h_limbs, out, out_limbs, params, c, sh.bytes, hs, nullptr, c + cells,
                  scratch_bytes - cells);
}

int set_error(int code, const char *msg) {
    snprintf(g_last_error, sizeof g_last_error, "%s", msg);
    if (getenv("TFT_DEBUG")) fprintf(stderr, "[tft] %s\n", g_last_error);
    return code;
}

}  // namespace tft

extern "C" {

int zx_mul_ss(const uint32_t *g, uint64_t len_g, uint32_t g_limbs, const uint32_t *h, uint64_t len_h,
              uint32_t h_limbs, uint32_t *out, uint32_t out_limbs, const tft_ss_params *params, void *ws,
              uint64_t ws_bytes, void *stream) {
    return ss_run(g, len_g, g_limbs, h, len_h, h_limbs, out, out_limbs, params, ws, ws_bytes,
                  static_cast<hipStream_t>(stream), nullptr);
}

int zx_mul_ss_timed(const uint32_t *g, uint64_t len_g, uint32_t g_limbs, const uint32_t *h, uint64_t len_h,
                    uint32_t h_limbs, uint32_t *out, uint32_t out_limbs, const tft_ss_params *params, void *ws,
                    uint64_t ws_bytes, void *stream, tft_ss_timing *timing) {
    if (!timing) return TFT_E_ARG;
    return ss_run(g, len_g, g_limbs, h, len_h, h_limbs, out, out_limbs, params, ws, ws_bytes,
                  static_cast<hipStream_t>(stream), timing);
}

// ---------------------------------------------------------------------------
// Schoenhage-Nussbaumer in (Z/mZ)[x] (Sect. 5.2)
// ---------------------------------------------------------------------------

struct SNShape {
    uint32_t K, l;
    uint64_t zg, zh, n, L, ws;
};

static int sn_shape(uint64_t len_g, uint64_t len_h, uint32_t log2K, SNShape *o) {
    if (len_g < 1 || len_h < 1 || log2K < 1 || log2K > 12) return TFT_E_ARG;
    const uint64_t K = 1ull << log2K, piece = K / 2;
    o->K = (uint32_t)K;
    o->zg = (len_g + piece - 1) / piece;
    o->zh = (len_h + piece - 1) / piece;
    o->n = o->zg + o->zh - 1;
    o->l = std::max<uint32_t>(1, log2u(o->n));
    o->L = 1ull << o->l;
    if (o->L > 2 * K) return TFT_E_ARG;
    o->ws = 2 * o->L * K * 8ull;
    return TFT_OK;
}

int zmx_mul_nussbaumer_workspace(uint64_t len_g, uint64_t len_h, uint32_t log2K, uint64_t *bytes) {
    if (!bytes) return TFT_E_ARG;
    SNShape sh;
    int st = sn_shape(len_g, len_h, log2K, &sh);
    if (st) return st;
    *bytes = sh.ws;
    return TFT_OK;
}

int zmx_mul_nussbaumer(const uint64_t *g, uint64_t len_g, const uint64_t *h, uint64_t len_h, uint64_t m,
                       uint32_t log2K, uint64_t *out, void *ws, uint64_t ws_bytes, void *stream) {
    if (!g || !h || !out) return TFT_E_ARG;
    SNShape sh;
    int st = sn_shape(len_g, len_h, log2K, &sh);
    if (st) return st;
    tft_ring ring{TFT_RING_NEGA, 0, sh.K, 0, m};
    st = check_ring(&ring);
    if (st) return st;
    if (!ws || ws_bytes < sh.ws) return TFT_E_WORKSPACE;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    uint64_t *A = static_cast<uint64_t *>(ws);
    uint64_t *B = A + sh.L * sh.K;
    hipError_t e = launch_nega_pack(sh.K, g, len_g, A, sh.zg, hs);
    if (e == hipSuccess) e = launch_nega_pack(sh.K, h, len_h, B, sh.zh, hs);
    if (e != hipSuccess) return dev_fail(e, "pack");
    st = plan_run(cached_plan(&ring, 0, sh.l, 0, sh.zg, sh.n, 0, nullptr), A, hs);
    if (st) return st;
    st = plan_run(cached_plan(&ring, 0, sh.l, 0, sh.zh, sh.n, 0, nullptr), B, hs);
    if (st) return st;
    e = launch_nega_pointwise(sh.K, m, sh.n, A, B, A, sh.l, hs);
    if (e != hipSuccess) return dev_fail(e, "pointwise");
    st = plan_run(cached_plan(&ring, 1, sh.l, 0, sh.n, sh.n, 0, nullptr), A, hs);
    if (st) return st;
    return hip_status(launch_nega_unpack(sh.K, m, A, sh.n, out, len_g + len_h - 1, hs));
}

// ---------------------------------------------------------------------------
// (Z/pZ)[x] by TFT / pointwise products / ITFT over Z/pZ (Sect. 2, Sect. 6)
// ---------------------------------------------------------------------------

static int zp_shape(uint64_t len_g, uint64_t len_h, uint32_t pad_rows, uint32_t *l, uint64_t *nt) {
    if (len_g < 1 || len_h < 1 || pad_rows > 1) return TFT_E_ARG;
    const uint64_t n = len_g + len_h - 1;
    const uint32_t lg = std::max<uint32_t>(1, log2u(n));
    if (lg > zp::ORD_LOG2) return TFT_E_ARG;
    uint64_t t = n;
    if (pad_rows) {  // whole rows of the paper's split (Sect. 6): L2 = 2^(l - floor(l/2))
        const uint64_t L2 = 1ull << (lg - lg / 2);
        t = (n + L2 - 1) / L2 * L2;
    }
    *l = lg;
    *nt = t;
    return TFT_OK;
}

int zpx_mul_ntt_workspace(uint64_t len_g, uint64_t len_h, uint64_t *bytes) {
    uint32_t l;
    uint64_t nt;
    if (!bytes) return TFT_E_ARG;
    int st = zp_shape(len_g, len_h, 0, &l, &nt);
    if (st) return st;
    *bytes = 2ull * (1ull << l) * 4ull;
    return TFT_OK;
}

int zpx_mul_ntt(const uint32_t *g, uint64_t len_g, const uint32_t *h, uint64_t len_h, uint32_t pad_rows,
                uint32_t *out, void *ws, uint64_t ws_bytes, void *stream) {
    if (!g || !h || !out) return TFT_E_ARG;
    uint32_t l;
    uint64_t nt;
    int st = zp_shape(len_g, len_h, pad_rows, &l, &nt);
    if (st) return st;
    const uint64_t L = 1ull << l, n = len_g + len_h - 1;
    if (!ws || ws_bytes < 2ull * L * 4ull) return TFT_E_WORKSPACE;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const tft_ring ring{TFT_RING_PRIME, 0, 0, 0, zp::P};
    uint32_t *A = static_cast<uint32_t *>(ws), *B = A + L;
    // cells beyond the operand lengths are never read (Sect. 3: they hold zeros)
    hipError_t e = hipMemcpyAsync(A, g, len_g * 4ull, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(B, h, len_h * 4ull, hipMemcpyDeviceToDevice, hs);
    if (e != hipSuccess) return dev_fail(e, "operand copy");
    st = plan_run(cached_plan(&ring, 0, l, 0, len_g, nt, 0, nullptr), A, hs);
    if (!st) st = plan_run(cached_plan(&ring, 0, l, 0, len_h, nt, 0, nullptr), B, hs);
    if (st) return st;
    e = launch_zp_pointwise(nt, A, B, A, l, hs);
    if (e != hipSuccess) return dev_fail(e, "pointwise");
    st = plan_run(cached_plan(&ring, 1, l, 0, nt, nt, 0, nullptr), A, hs);
    if (st) return st;
    return hip_status(hipMemcpyAsync(out, A, n * 4ull, hipMemcpyDeviceToDevice, hs), "output copy");
}

}  // extern "C"
