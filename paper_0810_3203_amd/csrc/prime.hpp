// Arithmetic in R = Z/pZ for the word-size prime p = 15 2^27 + 1 (the
// small-coefficient case of Sect. 6), shared by the host planner (twiddle
// tables) and the device kernels.
//
// theta = r^15 with r = 31, the smallest primitive root mod p, so theta has
// order exactly 2^27 = ord(theta): every power-of-two transform length up to
// 2^27 has its principal root omega_L = theta^(2^27 / L) (Sect. 2).
// Residues are uint32 in [0, p).  Products use Montgomery reduction with
// R = 2^32: mont(a, b) = a b / R mod p.  A value kept "in Montgomery form"
// is v R mod p, so mont(x, v R) = x v for a plain x.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define TFT_PHD __host__ __device__ __forceinline__
#else
#define TFT_PHD inline
#endif

namespace tft {
namespace zp {

constexpr uint32_t P = 15u * (1u << 27) + 1u;  // 2013265921
constexpr uint32_t ORD_LOG2 = 27;
constexpr uint32_t ORD = 1u << ORD_LOG2;
constexpr uint32_t ROOT = 31;  // smallest primitive root mod P

// -P^-1 mod 2^32 by Newton's iteration (x <- x (2 - P x) doubles the bits)
constexpr uint32_t neg_inv_p() {
    uint32_t x = 1;
    for (int i = 0; i < 5; ++i) x *= 2u - P * x;
    return 0u - x;
}
constexpr uint32_t PINV = neg_inv_p();
constexpr uint32_t R2 = (uint32_t)(((unsigned __int128)1 << 64) % P);  // R^2 mod P

// Reductions by the unsigned minimum: for v < 2P, v - P wraps around to a
// value above v exactly when v < P, so min(v, v - P) is v mod P.
TFT_PHD constexpr uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }
TFT_PHD constexpr uint32_t mont(uint32_t a, uint32_t b) {
    const uint64_t t = (uint64_t)a * b;
    const uint32_t m = (uint32_t)t * PINV;
    const uint32_t u = (uint32_t)((t + (uint64_t)m * P) >> 32);  // < 2P
    return umin(u, u - P);
}
TFT_PHD constexpr uint32_t to_mont(uint32_t a) { return mont(a, R2); }
TFT_PHD constexpr uint32_t from_mont(uint32_t a) { return mont(a, 1u); }
TFT_PHD constexpr uint32_t add(uint32_t a, uint32_t b) {
    const uint32_t s = a + b;  // < 2P < 2^32
    return umin(s, s - P);
}
// a - b wraps to at least 2^32 - P > P when a < b; adding P then brings it below P
TFT_PHD constexpr uint32_t sub(uint32_t a, uint32_t b) {
    const uint32_t d = a - b;
    return umin(d, d + P);
}
TFT_PHD constexpr uint32_t half(uint32_t a) { return (a + ((a & 1u) ? P : 0u)) >> 1; }

// b^e in Montgomery form, b given in Montgomery form
TFT_PHD constexpr uint32_t pow_m(uint32_t bm, uint64_t e) {
    uint32_t r = to_mont(1u);
    while (e) {
        if (e & 1u) r = mont(r, bm);
        bm = mont(bm, bm);
        e >>= 1;
    }
    return r;
}
constexpr uint32_t THETA_M = pow_m(to_mont(ROOT), 15);  // theta in Montgomery form

// theta^e (e taken mod ORD) in Montgomery form
TFT_PHD constexpr uint32_t theta_pow_m(uint64_t e) { return pow_m(THETA_M, e & (ORD - 1u)); }

}  // namespace zp
}  // namespace tft
