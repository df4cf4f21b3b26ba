// Device arithmetic in R = Z/(2^N+1), theta = 2 (Sect. 2 example ring; Sect. 5.1),
// organised for 64-wide wavefronts on gfx950.
//
// A residue is W = N/32 little-endian 32-bit limbs plus a top word (value =
// limbs + top*2^N, canonical in [0, 2^N]).  One element is processed by a
// "segment" of S lanes: limb k = r*S + l sits in lane l of row r, for rows
// r < R (W = S*R).  With W >= 64 a segment is the whole wave (S = 64,
// R = W/64); with W < 64 a wave holds 64/W segments of one row each, so
// 64/W base cases run side by side.
//
// Multi-limb addition resolves carries across the 64 lanes of a row with a
// carry-lookahead on wave masks (ballots): generate G (limb sum overflowed),
// propagate P (limb sum is all ones); the carries into the lanes are the bits
// of ((G|P) + G + cin) ^ P, computed on the scalar unit.  Rows are chained by
// the carry out of their last lane.  Subtraction is the same with borrows.
//
// Multiplication by theta^e = 2^e (the twiddles; Sect. 6 stores zeta as its
// exponent) is a cyclic rotation by t = e mod N bits with the wrapped part
// negated (2^N = -1), and a global sign when e >= N.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tft {

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ bool lane_bit(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }
__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

constexpr uint64_t seg_last_mask(int S) {
    uint64_t m = 0;
    for (int g = 0; g < 64 / S; ++g) m |= 1ull << (g * S + S - 1);
    return m;
}

template <int S_, int R_>
struct FermatSeg {
    static constexpr int S = S_;
    static constexpr int R = R_;
    static constexpr int W = S * R;
    static constexpr uint32_t N = 32u * W;
    static constexpr uint64_t LAST = seg_last_mask(S);
    static_assert(S == 64 || R == 1, "segments narrower than a wave hold one row");
    static_assert((W & (W - 1)) == 0, "W must be a power of two");

    uint32_t lane;  // 0..63
    uint32_t l;     // lane within the segment
    uint32_t g0;    // first lane of the segment

    __device__ FermatSeg() {
        lane = lane_id();
        l = lane & (S - 1);
        g0 = lane - l;
    }

    // carry (or borrow) value of this lane's segment held in a mask with bits at segment starts
    __device__ __forceinline__ uint32_t seg_bit(uint64_t c) const { return (uint32_t)((c >> g0) & 1ull); }

    __device__ __forceinline__ uint32_t resolve(uint32_t v, uint64_t G, uint64_t P, uint64_t &c, bool sub) const {
        const uint64_t Gm = G & ~LAST, Pm = P & ~LAST;
        const uint64_t X = (Gm | Pm) + Gm + c;
        const uint64_t C = X ^ Pm;  // carry (borrow) into each lane
        const uint64_t cout = (G | (P & C)) & LAST;
        c = cout >> (S - 1);
        const uint32_t ci = lane_bit(C) ? 1u : 0u;
        return sub ? v - ci : v + ci;
    }

    // one row of a chained addition a + b (+ carry in c); c becomes the carry out
    __device__ __forceinline__ uint32_t add_row(uint32_t a, uint32_t b, uint64_t &c) const {
        uint32_t s;
        const bool gen = __builtin_add_overflow(a, b, &s);
        return resolve(s, ballot(gen), ballot(s == 0xFFFFFFFFu), c, false);
    }

    // one row of a chained subtraction a - b (- borrow in c)
    __device__ __forceinline__ uint32_t sub_row(uint32_t a, uint32_t b, uint64_t &c) const {
        uint32_t d;
        const bool gen = __builtin_sub_overflow(a, b, &d);
        return resolve(d, ballot(gen), ballot(d == 0u), c, true);
    }

    // Add (sub = false) or subtract (sub = true) the 64-bit value hi:lo placed at
    // limb k0 of the segment's element x.  Returns the carry (borrow) out of
    // limb W-1 plus the part of hi that lands beyond it.  Rows are visited only
    // while a carry still moves.
    __device__ uint32_t prop(uint32_t *x, uint32_t lo, uint32_t hi, uint32_t k0, bool sub) const {
        if (ballot(lo != 0u || hi != 0u) == 0ull) return 0u;
        uint32_t over = (k0 + 1u >= (uint32_t)W) ? hi : 0u;
        if (k0 + 1u >= (uint32_t)W) hi = 0u;
        uint32_t r0 = 0, rhi = 0;
        if (S == 64) {
            r0 = uniform(k0) >> 6;
            rhi = uniform(hi != 0u ? k0 + 1u : k0) >> 6;
        }
        uint64_t c = 0;
        for (uint32_t r = r0; r < (uint32_t)R; ++r) {
            if (r > rhi && c == 0ull) break;
            const uint32_t k = r * S + l;
            const uint32_t add = (k == k0) ? lo : ((k == k0 + 1u) ? hi : 0u);
            const uint32_t v = x[k];
            x[k] = sub ? sub_row(v, add, c) : add_row(v, add, c);
        }
        return seg_bit(c) + over;
    }

    // Canonicalise in place: the element's value is Y + exc*2^N + corr*2^cbit
    // (Y = the W limbs of x, |corr| <= 2, small exc).  Writes the top word.
    __device__ void canon(uint32_t *x, uint32_t *top, int exc, int corr, uint32_t cbit) const {
        if (ballot(corr != 0) != 0ull) {
            const uint32_t k0 = cbit >> 5, sh = cbit & 31u;
            const uint64_t mag = (uint64_t)(uint32_t)(corr < 0 ? -corr : corr) << sh;
            const uint64_t mp = corr > 0 ? mag : 0ull, mn = corr < 0 ? mag : 0ull;
            exc += (int)prop(x, (uint32_t)mp, (uint32_t)(mp >> 32), k0, false);
            exc -= (int)prop(x, (uint32_t)mn, (uint32_t)(mn >> 32), k0, true);
        }
        // value = Y - exc (mod 2^N + 1)
        int o2 = 0;
        if (ballot(exc != 0) != 0ull) {
            const uint32_t ap = exc < 0 ? (uint32_t)(-exc) : 0u;
            const uint32_t an = exc > 0 ? (uint32_t)exc : 0u;
            o2 = (int)prop(x, ap, 0u, 0u, false) - (int)prop(x, an, 0u, 0u, true);
        }
        // value = Y' + o2*2^N = Y' - o2, with Y' <= 3 if o2 = 1 and Y' >= 2^N - 5 if o2 = -1
        uint32_t t = 0;
        if (ballot(o2 != 0) != 0ull) {
            const uint32_t y0 = x[0];
            if (o2 == 1) {
                if (y0 == 0u)
                    t = 1u;
                else if (l == 0)
                    x[0] = y0 - 1u;
            } else if (o2 == -1) {
                if (y0 == 0xFFFFFFFFu) {
                    t = 1u;
                    for (uint32_t r = 0; r < (uint32_t)R; ++r) x[r * S + l] = 0u;
                } else if (l == 0) {
                    x[0] = y0 + 1u;
                }
            }
        }
        if (l == 0) *top = t;
    }
};

// Rotation parameters of a multiplication by 2^e, 0 <= e < 2N.
template <class F>
struct Rot {
    uint32_t t;     // e mod N: bits rotated
    uint32_t q;     // t / 32
    uint32_t rb;    // t % 32
    uint32_t qp;    // q + (rb != 0)
    uint32_t c;     // (32 - rb) % 32
    bool neg;       // e >= N: 2^e = -2^t

    __device__ __forceinline__ explicit Rot(uint32_t e) {
        neg = e >= F::N;
        t = neg ? e - F::N : e;
        q = t >> 5;
        rb = t & 31u;
        qp = q + (rb != 0u ? 1u : 0u);
        c = (32u - rb) & 31u;
    }
    // limb k of x rotated left by t bits within N bits
    __device__ __forceinline__ uint32_t read(const uint32_t *x, uint32_t k) const {
        const uint32_t lo = x[(k - qp) & (uint32_t)(F::W - 1)];
        const uint32_t hi = x[(k - qp + 1u) & (uint32_t)(F::W - 1)];
        return __builtin_amdgcn_alignbit(hi, lo, c);
    }
    // bits of limb k below t: the part of x*2^t that wrapped past 2^N
    __device__ __forceinline__ uint32_t low(uint32_t k) const {
        return k < q ? 0xFFFFFFFFu : (k == q ? ((1u << rb) - 1u) : 0u);
    }
};

// The base cases of Alg. 1 and Alg. 2 on canonical cells of LDS.
template <class F>
struct FermatOps : F {
    using F::R;
    using F::S;
    using F::W;

    // D = sgn * (A - B) row by row (D kept in registers), where for
    // 2^t (x0 - x1) = (Lo0 - Hi0) - (Lo1 - Hi1) the merged words are
    // A = Lo0 | Hi1 and B = Lo1 | Hi0 (Lo, Hi: the bits of the rotation at
    // and above t, and below t).  x1 == nullptr means x1 = 0.
    __device__ __forceinline__ void rot_diff(const uint32_t *x0, const uint32_t *x1, const Rot<F> &rt,
                                             uint32_t (&D)[R], uint64_t &bD) const {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = (uint32_t)r * S + this->l;
            const uint32_t r0 = rt.read(x0, k);
            const uint32_t r1 = x1 ? rt.read(x1, k) : 0u;
            const uint32_t lo = rt.low(k);
            const uint32_t A = (r1 & lo) | (r0 & ~lo);
            const uint32_t B = (r0 & lo) | (r1 & ~lo);
            D[r] = rt.neg ? this->sub_row(B, A, bD) : this->sub_row(A, B, bD);
        }
    }

    // TFT z=2 n=2: (x0, x1) <- (x0 + x1, 2^e (x0 - x1))
    __device__ void t22(uint32_t *x0, uint32_t *x1, uint32_t *tp0, uint32_t *tp1, uint32_t e) const {
        const Rot<F> rt(e);
        uint32_t D[R];
        uint64_t bD = 0, c0 = 0;
        rot_diff(x0, x1, rt, D, bD);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = (uint32_t)r * S + this->l;
            const uint32_t y = this->add_row(x0[k], x1[k], c0);
            x0[k] = y;
            x1[k] = D[r];
        }
        const int t0 = (int)*tp0, t1 = (int)*tp1;
        const int sg = rt.neg ? -1 : 1;
        this->canon(x0, tp0, (int)this->seg_bit(c0) + t0 + t1, 0, 0u);
        this->canon(x1, tp1, -(int)this->seg_bit(bD), sg * (t1 - t0), rt.t);
    }

    // TFT z=1 n=2: x1 <- 2^e x0
    __device__ void t21(uint32_t *x0, uint32_t *x1, uint32_t *tp0, uint32_t *tp1, uint32_t e) const {
        const Rot<F> rt(e);
        uint32_t D[R];
        uint64_t bD = 0;
        rot_diff(x0, nullptr, rt, D, bD);
#pragma unroll
        for (int r = 0; r < R; ++r) x1[(uint32_t)r * S + this->l] = D[r];
        const int t0 = (int)*tp0;
        const int sg = rt.neg ? -1 : 1;
        this->canon(x1, tp1, -(int)this->seg_bit(bD), -sg * t0, rt.t);
    }

    // x0 <- x0 + x1
    __device__ void add2(uint32_t *x0, const uint32_t *x1, uint32_t *tp0, const uint32_t *tp1) const {
        uint64_t c0 = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = (uint32_t)r * S + this->l;
            x0[k] = this->add_row(x0[k], x1[k], c0);
        }
        this->canon(x0, tp0, (int)this->seg_bit(c0) + (int)*tp0 + (int)*tp1, 0, 0u);
    }

    // x0 <- 2 x0 - x1 (x1 == nullptr: x0 <- 2 x0)
    __device__ void dbl_sub(uint32_t *x0, const uint32_t *x1, uint32_t *tp0, const uint32_t *tp1) const {
        uint64_t bu = 0, c0 = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = (uint32_t)r * S + this->l;
            const uint32_t a = x0[k];
            const uint32_t u = x1 ? this->sub_row(a, x1[k], bu) : a;
            x0[k] = this->add_row(a, u, c0);
        }
        const int t0 = (int)*tp0, t1 = x1 ? (int)*tp1 : 0;
        this->canon(x0, tp0, (int)this->seg_bit(c0) - (int)this->seg_bit(bu) + 2 * t0 - t1, 0, 0u);
    }

    // ITFT n=2: (x0, x1) <- (x0 + 2^-e x1, x0 - 2^-e x1); einv = -e mod 2N
    __device__ void i2(uint32_t *x0, uint32_t *x1, uint32_t *tp0, uint32_t *tp1, uint32_t einv) const {
        const Rot<F> rt(einv);
        uint32_t V[R];
        uint64_t bV = 0, c0 = 0, b1 = 0;
        rot_diff(x1, nullptr, rt, V, bV);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = (uint32_t)r * S + this->l;
            const uint32_t a = x0[k];
            x0[k] = this->add_row(a, V[r], c0);
            x1[k] = this->sub_row(a, V[r], b1);
        }
        const int t0 = (int)*tp0, t1 = (int)*tp1;
        const int sg = rt.neg ? -1 : 1;
        const int bv = (int)this->seg_bit(bV);
        this->canon(x0, tp0, (int)this->seg_bit(c0) + t0 - bv, -sg * t1, rt.t);
        this->canon(x1, tp1, -(int)this->seg_bit(b1) + t0 + bv, sg * t1, rt.t);
    }

    // ITFT n=1 f=1: (x0, x1) <- (2 x0 - x1, 2^e (x0 - x1)); z=1: x1 taken as 0
    __device__ void i1f1(uint32_t *x0, uint32_t *x1, uint32_t *tp0, uint32_t *tp1, uint32_t e, bool z2) const {
        const Rot<F> rt(e);
        uint32_t D[R];
        uint64_t bD = 0, bu = 0, c0 = 0;
        rot_diff(x0, z2 ? x1 : nullptr, rt, D, bD);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = (uint32_t)r * S + this->l;
            const uint32_t a = x0[k];
            const uint32_t u = z2 ? this->sub_row(a, x1[k], bu) : a;
            x0[k] = this->add_row(a, u, c0);
            x1[k] = D[r];
        }
        const int t0 = (int)*tp0, t1 = z2 ? (int)*tp1 : 0;
        const int sg = rt.neg ? -1 : 1;
        this->canon(x0, tp0, (int)this->seg_bit(c0) - (int)this->seg_bit(bu) + 2 * t0 - t1, 0, 0u);
        this->canon(x1, tp1, -(int)this->seg_bit(bD), sg * (t1 - t0), rt.t);
    }

    // x0 <- 2^e x0 in place
    __device__ void scale(uint32_t *x0, uint32_t *tp0, uint32_t e) const {
        const Rot<F> rt(e);
        uint32_t V[R];
        uint64_t bV = 0;
        rot_diff(x0, nullptr, rt, V, bV);
#pragma unroll
        for (int r = 0; r < R; ++r) x0[(uint32_t)r * S + this->l] = V[r];
        const int t0 = (int)*tp0;
        const int sg = rt.neg ? -1 : 1;
        this->canon(x0, tp0, -(int)this->seg_bit(bV), -sg * t0, rt.t);
    }
};

}  // namespace tft
