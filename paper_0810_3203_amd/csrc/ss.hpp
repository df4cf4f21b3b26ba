// Shape of a Schoenhage-Strassen product in Z[x] over R = Z/(2^N+1) (Sect. 5.1),
// with k >= 1 coefficients bundled per ring element: the operands become
// polynomials in X = x^k whose coefficients are k-slot integers (slot width ws
// limbs, wide enough for any output coefficient); a product cell then holds
// 2k-1 slots, so N >= 32 (2k-1) ws, and L = 2^l must divide 2N.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tft.h"

namespace tft {

struct SSShape {
    uint32_t N, W, l, k, ws;
    uint64_t zg, zh, n, L, bytes;
    uint64_t nt;    // truncation of the transforms: n, or n rounded up to whole top-level rows
    uint32_t s;     // twist of TFT(g), TFT(h): zeta = theta^s, s < 2N; the ITFT takes zeta^2
    uint64_t bits;  // bound on the bits of an output coefficient
};

// Leaf size (log2 cells) of one product's transforms when the caller leaves it
// open: about two leaf jobs per compute unit per pass for long transforms, two
// half-length passes for short ones, never beyond what fits the LDS.
uint32_t ss_leaf_log2(uint32_t N, uint32_t l);

inline uint32_t ss_log2u(uint64_t v) {
    uint32_t l = 0;
    while ((1ull << l) < v) l++;
    return l;
}

inline int ss_shape(uint64_t len_g, uint32_t g_limbs, uint64_t len_h, uint32_t h_limbs, const tft_ss_params *p,
                    SSShape *o) {
    if (len_g < 1 || len_h < 1 || g_limbs < 1 || h_limbs < 1) return TFT_E_ARG;
    const uint32_t k = (p && p->k) ? p->k : 1u;
    if (k > 64) return TFT_E_ARG;
    const uint64_t bits = 32ull * (g_limbs + h_limbs) + ss_log2u(len_g < len_h ? len_g : len_h);
    const uint64_t ws = (bits + 31) / 32;
    const uint64_t zg = (len_g + k - 1) / k, zh = (len_h + k - 1) / k;
    const uint64_t n = zg + zh - 1;
    const uint32_t l = (p && p->l) ? p->l : (ss_log2u(n) < 1 ? 1u : ss_log2u(n));
    if (l > 24 || (1ull << l) < n) return TFT_E_ARG;
    const uint64_t L = 1ull << l;
    const uint64_t need = (k == 1) ? ws : (2ull * k - 1) * ws;  // limbs a product cell needs
    uint64_t W;
    if (p && p->N) {
        if (p->N % 32) return TFT_E_RING;
        W = p->N / 32;
        if ((W & (W - 1)) || W > 4096) return TFT_E_RING;
        if ((64 * W) % L) return TFT_E_RING;
        if (W < need) return TFT_E_RANGE;
    } else {
        W = 1;
        while (W < need || 64 * W < L) W <<= 1;
        if (W > 4096) return TFT_E_UNSUPPORTED;
    }
    o->N = (uint32_t)(32 * W);
    o->W = (uint32_t)W;
    o->l = l;
    o->k = k;
    o->ws = (uint32_t)ws;
    o->zg = zg;
    o->zh = zh;
    o->n = n;
    o->nt = n;
    o->s = p ? (uint32_t)(p->zeta_exp % (2ull * W * 32)) : 0u;
    if (p && p->pad_rows) {
        if (p->pad_rows > 1) return TFT_E_ARG;
        // rows of the top split (Alg. 1, Alg. 2): L2 = 2^(l - l1)
        const uint32_t t = p->split.top_l1;
        const uint32_t l1 = t == TFT_SPLIT_DC ? 1u : (t && t < l) ? t : l / 2;
        const uint64_t L2 = 1ull << (l - l1);
        o->nt = (n + L2 - 1) / L2 * L2;
    }
    o->L = L;
    o->bytes = 2 * L * (W + 1) * 4ull;
    o->bits = bits;
    return TFT_OK;
}

// A product run from one device scratch area: its cell arrays first, then the
// descriptors of its three transform plans (copied in on the stream).
// ss_scratch_bytes: the area a request needs (host work: builds the plans).
// ss_scratch_run: TFT_E_WORKSPACE if the request needs more than scratch_bytes.
int ss_scratch_bytes(uint64_t len_g, uint32_t g_limbs, uint64_t len_h, uint32_t h_limbs, uint32_t out_limbs,
                     const tft_ss_params *params, uint64_t *bytes);
int ss_scratch_run(const uint32_t *g, uint64_t len_g, uint32_t g_limbs, const uint32_t *h, uint64_t len_h,
                   uint32_t h_limbs, uint32_t *out, uint32_t out_limbs, const tft_ss_params *params, void *scratch,
                   uint64_t scratch_bytes, hipStream_t hs);
// Sets the message tft_last_error returns; returns code.
int set_error(int code, const char *msg);

}  // namespace tft
