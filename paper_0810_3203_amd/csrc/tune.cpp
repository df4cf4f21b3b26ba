// Choosing the parameters of a Schoenhage-Strassen product (bundling factor k,
// hence ring size and transform length, and the top Bailey split of Alg. 1/2):
// the candidate set, a fixed default rule, the features the cost model reads,
// exhaustive timing of the candidates, and selection by the cost model.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/tft.h"
#include "kernels.hpp"
#include "plan.hpp"
#include "ss.hpp"

using namespace tft;

namespace {

const uint32_t kKs[] = {1, 2, 4, 8, 16, 32};

uint32_t leaf_max(uint32_t W) {
    const uint64_t cap = lds_budget_bytes() / fermat_lds_cell_bytes(W);
    uint32_t lg = 0;
    while ((2ull << lg) <= cap) lg++;
    return std::min<uint32_t>(lg, 11);
}

std::vector<tft_ss_params> candidates(uint64_t len_g, uint32_t g_limbs, uint64_t len_h, uint32_t h_limbs) {
    std::vector<tft_ss_params> out;
    // p, p with n padded to whole rows when that changes the truncation, and
    // each of those with the forward twist zeta = theta^(3N/2) (tft_ss_params)
    auto push = [&](tft_ss_params p) {
        SSShape sh;
        if (ss_shape(len_g, g_limbs, len_h, h_limbs, &p, &sh)) return;
        const uint32_t twist = 3u * (32u * sh.W) / 2u;
        auto both = [&](tft_ss_params q) {
            out.push_back(q);
            q.zeta_exp = twist;
            out.push_back(q);
        };
        both(p);
        p.pad_rows = 1;
        SSShape sp;
        if (!ss_shape(len_g, g_limbs, len_h, h_limbs, &p, &sp) && sp.nt != sp.n) both(p);
    };
    for (uint32_t k : kKs) {
        tft_ss_params p{};
        p.k = k;
        SSShape sh;
        if (ss_shape(len_g, g_limbs, len_h, h_limbs, &p, &sh)) continue;
        if (sh.n < 2 && k > 1) continue;  // larger k cannot shrink a single-cell product
        push(p);
        // second split: one column pass of leaf size, then rows of the rest
        const uint32_t lm = leaf_max(sh.W);
        if (sh.l > lm) {
            const uint32_t top = sh.l - lm;
            if (top != sh.l / 2 && top >= 1) {
                p.split.top_l1 = top;
                push(p);
            }
        }
        if (sh.n == 1) break;
    }
    return out;
}

float log2f_safe(double v) { return (float)std::log2(std::max(v, 1.0)); }

}  // namespace

extern "C" {

int tft_ss_candidates(uint64_t len_g, uint32_t g_limbs, uint64_t len_h, uint32_t h_limbs, tft_ss_params *out,
                      uint32_t cap, uint32_t *count) {
    if (!count) return TFT_E_ARG;
    SSShape sh;
    int st = ss_shape(len_g, g_limbs, len_h, h_limbs, nullptr, &sh);
    if (st && st != TFT_E_UNSUPPORTED) return st;
    const auto c = candidates(len_g, g_limbs, len_h, h_limbs);
    *count = (uint32_t)c.size();
    if (c.empty()) return TFT_E_UNSUPPORTED;
    if (out) {
        if (cap < c.size()) return TFT_E_ARG;
        std::copy(c.begin(), c.end(), out);
    }
    return TFT_OK;
}

int tft_ss_default_params(uint64_t len_g, uint32_t g_limbs, uint64_t len_h, uint32_t h_limbs,
                          tft_ss_params *out) {
    if (!out) return TFT_E_ARG;
    uint64_t best = 0;
    std::vector<std::pair<uint32_t, uint64_t>> fp;  // (k, footprint bytes)
    for (uint32_t k : kKs) {
        tft_ss_params p{};
        p.k = k;
        SSShape sh;
        if (ss_shape(len_g, g_limbs, len_h, h_limbs, &p, &sh)) continue;
        fp.emplace_back(k, sh.bytes);
        if (!best || sh.bytes < best) best = sh.bytes;
        if (sh.n == 1) break;
    }
    if (fp.empty()) return TFT_E_UNSUPPORTED;
    // smallest k whose cell-array footprint is within 5/4 of the smallest one
    for (const auto &kv : fp)
        if (4 * kv.second <= 5 * best) {
            *out = tft_ss_params{};
            out->k = kv.first;
            return TFT_OK;
        }
    return TFT_E_UNSUPPORTED;
}

int tft_ss_features(uint64_t len_g, uint32_t g_limbs, uint64_t len_h, uint32_t h_limbs, const tft_ss_params *p,
                    float *feat) {
    if (!feat) return TFT_E_ARG;
    SSShape sh;
    int st = ss_shape(len_g, g_limbs, len_h, h_limbs, p, &sh);
    if (st) return st;
    const bool dc = p && p->split.top_l1 == TFT_SPLIT_DC;
    const uint32_t top = dc ? 1 : (p && p->split.top_l1 && p->split.top_l1 < sh.l) ? p->split.top_l1 : sh.l / 2;
    const double L = (double)sh.L, W = (double)sh.W;
    // leaf passes of the three transforms as zx_mul_ss plans them
    const uint32_t leaf = (p && p->split.leaf_log2) ? std::min(leaf_max(sh.W), p->split.leaf_log2)
                                                    : ss_leaf_log2(sh.N, sh.l);
    const uint32_t tsplit = p ? p->split.top_l1 : 0;
    const uint32_t pt = std::max(schedule_pass_count(0, sh.l, sh.zg, sh.nt, 0, leaf, tsplit),
                                 schedule_pass_count(0, sh.l, sh.zh, sh.nt, 0, leaf, tsplit));
    const uint32_t pi = schedule_pass_count(1, sh.l, sh.nt, sh.nt, 0, leaf, tsplit);
    const double passes = 2.0 * pt + pi;
    float f[TFT_SS_FEATURES] = {
        log2f_safe((double)len_g) / 16.0f,
        log2f_safe((double)len_h) / 16.0f,
        log2f_safe((double)(g_limbs + h_limbs)) / 8.0f,
        log2f_safe((double)sh.k) / 8.0f,
        (float)sh.l / 16.0f,
        log2f_safe(W) / 12.0f,
        (float)((double)sh.nt / L),
        log2f_safe((double)sh.bytes) / 32.0f,
        log2f_safe((double)sh.nt * W * W) / 40.0f,           // schoolbook pointwise limb products
        log2f_safe((double)sh.bytes * passes / 3.0) / 36.0f, // bytes moved by the transform passes
        (float)pt / 8.0f,                                     // leaf passes of one TFT
        (float)top / (float)sh.l,                             // share of the top split in the columns
        (float)pi / 32.0f,                                    // leaf passes of the ITFT
        (float)(sh.nt != sh.n ? 1 : 0),                       // n padded to whole rows
        (float)(sh.s != 0u ? 1 : 0),                          // forward twist zeta != 1
    };
    std::copy(f, f + TFT_SS_FEATURES, feat);
    return TFT_OK;
}

int tft_ss_time(const tft_zx_request *req, const tft_ss_params *cands, uint32_t ncand, uint32_t reps, void *ws,
                uint64_t ws_bytes, void *stream, float *ms, uint32_t *best) {
    if (!req || !cands || !ncand || !ms || reps < 1 || reps > 1000) return TFT_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<hipEvent_t> ev(2 * reps);
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) return TFT_E_DEVICE;
    int rc = TFT_OK;
    for (uint32_t c = 0; c < ncand && !rc; c++) {
        // one untimed run builds and uploads the plans
        rc = zx_mul_ss(req->g, req->len_g, req->g_limbs, req->h, req->len_h, req->h_limbs, req->out, req->out_limbs,
                       &cands[c], ws, ws_bytes, stream);
        for (uint32_t r = 0; r < reps && !rc; r++) {
            if (hipEventRecord(ev[2 * r], st) != hipSuccess) rc = TFT_E_DEVICE;
            if (!rc)
                rc = zx_mul_ss(req->g, req->len_g, req->g_limbs, req->h, req->len_h, req->h_limbs, req->out,
                               req->out_limbs, &cands[c], ws, ws_bytes, stream);
            if (!rc && hipEventRecord(ev[2 * r + 1], st) != hipSuccess) rc = TFT_E_DEVICE;
        }
        if (!rc && hipEventSynchronize(ev[2 * reps - 1]) != hipSuccess) rc = TFT_E_DEVICE;
        if (!rc) {
            std::vector<float> t(reps);
            for (uint32_t r = 0; r < reps; r++) (void)hipEventElapsedTime(&t[r], ev[2 * r], ev[2 * r + 1]);
            std::sort(t.begin(), t.end());
            ms[c] = t[reps / 2];
        }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (rc) return rc;
    if (best) {
        uint32_t b = 0;
        for (uint32_t c = 1; c < ncand; c++)
            if (ms[c] < ms[b]) b = c;  // ties keep the smaller index
        *best = b;
    }
    return TFT_OK;
}

int tft_mlp_choose_ss(tft_mlp *mlp, tft_zx_request *reqs, uint32_t count, void *stream) {
    if (!mlp || (!reqs && count)) return TFT_E_ARG;
    std::vector<float> feat;
    std::vector<tft_ss_params> cand;
    std::vector<uint32_t> first(count + 1, 0);
    for (uint32_t i = 0; i < count; i++) {
        first[i] = (uint32_t)cand.size();
        const tft_zx_request &r = reqs[i];
        for (const tft_ss_params &p : candidates(r.len_g, r.g_limbs, r.len_h, r.h_limbs)) {
            float f[TFT_SS_FEATURES];
            if (tft_ss_features(r.len_g, r.g_limbs, r.len_h, r.h_limbs, &p, f)) continue;
            feat.insert(feat.end(), f, f + TFT_SS_FEATURES);
            cand.push_back(p);
        }
    }
    first[count] = (uint32_t)cand.size();
    if (cand.empty()) return TFT_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    float *dx = nullptr, *dy = nullptr;
    const size_t nc = cand.size();
    if (hipMalloc(&dx, feat.size() * sizeof(float)) != hipSuccess) return TFT_E_DEVICE;
    if (hipMalloc(&dy, nc * sizeof(float)) != hipSuccess) {
        (void)hipFree(dx);
        return TFT_E_DEVICE;
    }
    std::vector<float> y(nc);
    int rc = hipMemcpyAsync(dx, feat.data(), feat.size() * sizeof(float), hipMemcpyHostToDevice, st) == hipSuccess
                 ? TFT_OK
                 : TFT_E_DEVICE;
    if (!rc) rc = tft_mlp_forward(mlp, dx, (uint32_t)nc, dy, stream);
    if (!rc && hipMemcpyAsync(y.data(), dy, nc * sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = TFT_E_DEVICE;
    if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = TFT_E_DEVICE;
    (void)hipFree(dx);
    (void)hipFree(dy);
    if (rc) return rc;
    for (uint32_t i = 0; i < count; i++) {
        if (first[i] == first[i + 1]) continue;
        uint32_t b = first[i];
        for (uint32_t c = first[i] + 1; c < first[i + 1]; c++)
            if (y[c] < y[b]) b = c;
        reqs[i].params = cand[b];
    }
    return TFT_OK;
}

}  // extern "C"
