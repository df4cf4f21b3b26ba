// Device arithmetic in R = Z/(2^N+1), theta = 2 (Sect. 2 example ring; Sect. 5.1),
// organised for 64-wide wavefronts on gfx950.
//
// A residue is W = N/32 little-endian 32-bit limbs plus a top word (value =
// limbs + top*2^N, canonical in [0, 2^N]).  One element belongs to a segment
// of S lanes; lane l of the segment holds the C consecutive limbs
// [l*C, (l+1)*C) in registers (W = S*C).  With W >= 64 a segment is the whole
// wave (S = 64, C = W/64); with W < 64 a wave holds 64/W one-limb segments, so
// 64/W base cases run side by side.
//
// Addition and subtraction run the limb chain inside each lane (v_addc /
// v_subb with the carry in VCC), then settle the lane carry-outs: a lane's
// carry enters the next lane's chunk, repeated while a carry still moves
// (once for random data; a run of all-ones chunks takes one round per lane).
//
// Multiplication by 2^e (every twiddle; Sect. 6 keeps zeta as its exponent)
// is a rotation by t = e mod N bits with the bits that pass 2^N negated
// (2^N = -1), and a global sign when e >= N.  It reads the element from LDS
// at rotated addresses.  In LDS an element is stored transposed: limb k at
// position (k mod C) S + k / C, so that the S lanes reading limb j of their
// chunks read S consecutive words (distinct banks) at a fixed offset j S.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace tft {

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ bool lane_bit(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }
__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint32_t addc(uint32_t a, uint32_t b, uint32_t &c) {
    uint32_t co;
    const uint32_t r = __builtin_addc(a, b, c, &co);
    c = co;
    return r;
}
__device__ __forceinline__ uint32_t subb(uint32_t a, uint32_t b, uint32_t &c) {
    uint32_t co;
    const uint32_t r = __builtin_subc(a, b, c, &co);
    c = co;
    return r;
}

constexpr uint64_t seg_mask(int S, int off) {
    uint64_t m = 0;
    for (int g = 0; g < 64 / S; ++g) m |= 1ull << (g * S + off);
    return m;
}

template <int S_, int C_>
struct FChunk {
    static constexpr int S = S_;
    static constexpr int C = C_;
    static constexpr int W = S * C;
    static constexpr uint32_t N = 32u * W;
    static constexpr int ESZ = W;  // LDS dwords per element
    static constexpr uint64_t FIRST = seg_mask(S, 0);
    static constexpr uint64_t LAST = seg_mask(S, S - 1);
    static_assert(S == 64 || C == 1, "segments narrower than a wave hold one limb per lane");
    static_assert((W & (W - 1)) == 0 && (C & (C - 1)) == 0, "powers of two");

    uint32_t lane;  // 0..63
    uint32_t l;     // lane within the segment
    uint32_t g0;    // first lane of the segment

    __device__ FChunk() {
        lane = lane_id();
        l = lane & (S - 1);
        g0 = lane - l;
    }

    // LDS position of limb k of an element
    __device__ static __forceinline__ uint32_t addr(uint32_t k) { return (k % C) * S + k / C; }

    __device__ __forceinline__ uint32_t seg_bit(uint64_t m, int off) const {
        return (uint32_t)((m >> (g0 + off)) & 1ull);
    }

    __device__ __forceinline__ void ld(const uint32_t *x, uint32_t (&v)[C]) const {
#pragma unroll
        for (int j = 0; j < C; ++j) v[j] = x[j * S + l];
    }
    __device__ __forceinline__ void st(uint32_t *x, const uint32_t (&v)[C]) const {
#pragma unroll
        for (int j = 0; j < C; ++j) x[j * S + l] = v[j];
    }

    // Carry (borrow) cy out of each lane's chunk enters the next lane; repeat
    // while carries move.  Returns 1 if the segment's element overflowed
    // (carry or borrow out of limb W-1).
    __device__ __forceinline__ uint32_t settle(uint32_t (&s)[C], uint32_t cy, bool sub) const {
        uint64_t G = ballot(cy != 0u);
        uint64_t over = G & LAST;
        uint64_t Cm = (G << 1) & ~FIRST;
        while (Cm != 0ull) {
            uint32_t c = lane_bit(Cm) ? 1u : 0u;
            if (sub) {
#pragma unroll
                for (int j = 0; j < C; ++j) s[j] = subb(s[j], 0u, c);
            } else {
#pragma unroll
                for (int j = 0; j < C; ++j) s[j] = addc(s[j], 0u, c);
            }
            G = ballot(c != 0u);
            over |= G & LAST;
            Cm = (G << 1) & ~FIRST;
        }
        return seg_bit(over, S - 1);
    }

    // s = a + b; returns the carry out of the element (0/1)
    __device__ __forceinline__ uint32_t add(uint32_t (&s)[C], const uint32_t (&a)[C], const uint32_t (&b)[C]) const {
        uint32_t c = 0;
#pragma unroll
        for (int j = 0; j < C; ++j) s[j] = addc(a[j], b[j], c);
        return settle(s, c, false);
    }
    // s = a - b; returns the borrow out of the element (0/1)
    __device__ __forceinline__ uint32_t sub(uint32_t (&s)[C], const uint32_t (&a)[C], const uint32_t (&b)[C]) const {
        uint32_t c = 0;
#pragma unroll
        for (int j = 0; j < C; ++j) s[j] = subb(a[j], b[j], c);
        return settle(s, c, true);
    }

    // s += mag * 2^bit (SUB: s -= ...), mag small, 0 <= bit < N; returns the
    // carry (borrow) out of the element including the part of mag 2^bit that
    // lies at or beyond 2^N.
    template <bool SUB>
    __device__ uint32_t add_at_mag(uint32_t (&s)[C], uint32_t mag, uint32_t bit) const {
        const uint64_t m64 = (uint64_t)mag << (bit & 31u);
        const uint32_t k0 = bit >> 5;
        uint32_t lo = (uint32_t)m64, hi = (uint32_t)(m64 >> 32);
        const uint32_t hover = (k0 + 1u >= (uint32_t)W) ? hi : 0u;
        if (hover) hi = 0u;
        uint32_t c = 0;
        if (ballot(k0 != 0u || hi != 0u) == 0ull) {
            // every segment adds at limb 0 only: lane 0 of the segment, limb 0
            const uint32_t a0 = (l == 0u) ? lo : 0u;
            s[0] = SUB ? subb(s[0], a0, c) : addc(s[0], a0, c);
            if (ballot(c != 0u) == 0ull) return hover;
#pragma unroll
            for (int j = 1; j < C; ++j) s[j] = SUB ? subb(s[j], 0u, c) : addc(s[j], 0u, c);
        } else {
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const uint32_t k = l * C + j;
                const uint32_t a = (k == k0) ? lo : ((k == k0 + 1u) ? hi : 0u);
                s[j] = SUB ? subb(s[j], a, c) : addc(s[j], a, c);
            }
        }
        return settle(s, c, SUB) + hover;
    }

    // s += v * 2^bit (|v| small); returns the overflow: +1 carry out of the
    // element, -1 borrow out, 0 none.
    __device__ int add_at(uint32_t (&s)[C], int v, uint32_t bit) const {
        if (ballot(v < 0) == 0ull) return (int)add_at_mag<false>(s, (uint32_t)v, bit);
        if (ballot(v > 0) == 0ull) return -(int)add_at_mag<true>(s, (uint32_t)(-v), bit);
        // segments of one wave disagree in sign: positive parts, then negative parts
        const int o = (int)add_at_mag<false>(s, v > 0 ? (uint32_t)v : 0u, bit);
        return o - (int)add_at_mag<true>(s, v < 0 ? (uint32_t)(-v) : 0u, bit);
    }

    // Canonicalise s in place: the element's value is s + exc*2^N + corr*2^cbit
    // (small exc, |corr| <= 2).  Returns the top word.
    __device__ uint32_t canon(uint32_t (&s)[C], int exc, int corr, uint32_t cbit) const {
        if (ballot(corr != 0) != 0ull) exc += add_at(s, corr, cbit);
        // value = s - exc (mod 2^N + 1)
        int o2 = 0;
        if (ballot(exc != 0) != 0ull) o2 = add_at(s, -exc, 0u);
        // value = s + o2 2^N = s - o2; s <= 5 when o2 = 1, s >= 2^N - 6 when o2 = -1
        uint32_t top = 0;
        if (ballot(o2 != 0) != 0ull) {
            const uint32_t y0 = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(g0 * 4u), (int)s[0]);
            if (o2 == 1) {
                if (y0 == 0u)
                    top = 1u;
                else if (l == 0u)
                    s[0] = y0 - 1u;
            } else if (o2 == -1) {
                if (y0 == 0xFFFFFFFFu) {
                    top = 1u;
#pragma unroll
                    for (int j = 0; j < C; ++j) s[j] = 0u;
                } else if (l == 0u) {
                    s[0] = y0 + 1u;
                }
            }
        }
        return top;
    }
};

// Rotation parameters of a multiplication by 2^e, 0 <= e < 2N.
template <class F>
struct Rot {
    uint32_t t;   // e mod N: bits rotated
    uint32_t q;   // t / 32
    uint32_t pm;  // (1 << (t % 32)) - 1: wrapped bits of limb q
    uint32_t qp;  // q + (t % 32 != 0)
    uint32_t c;   // (32 - t % 32) % 32
    bool neg;     // e >= N: 2^e = -2^t
    int sg;       // -1 if neg else 1

    __device__ __forceinline__ explicit Rot(uint32_t e) {
        neg = e >= F::N;
        sg = neg ? -1 : 1;
        t = neg ? e - F::N : e;
        q = t >> 5;
        const uint32_t rb = t & 31u;
        pm = (1u << rb) - 1u;
        qp = q + (rb != 0u ? 1u : 0u);
        c = (32u - rb) & 31u;
    }
};

// Per-lane masks of a rotation: limb j of the lane's chunk takes its bits
// below position t (the wrapped part) from mask low(j) = all ones for j < jq,
// the partial mask pm for j = jq, zero above, with jq = q - l*C.  Built once
// per operation as two bit sets, then one sign-extending bit extract and one
// and-or per limb (no compare/select through lane masks).
template <int C>
struct RotMask {
    using B = typename std::conditional<(C > 32), uint64_t, uint32_t>::type;
    B lt, eq;  // bit j: j < jq; j == jq
    uint32_t pm;

    __device__ __forceinline__ RotMask(int jq, uint32_t pm_) : pm(pm_) {
        constexpr int NB = C > 32 ? 64 : 32;
        lt = jq >= C ? ~B(0) : (jq <= 0 ? B(0) : ((B(1) << jq) - B(1)));
        eq = (jq >= 0 && jq < C) ? (B(1) << jq) : B(0);
        (void)NB;
    }
    template <int J>
    __device__ __forceinline__ static uint32_t ext(B v) {  // 0 or all ones from bit J
        if constexpr (C > 32) {
            const uint32_t w = J < 32 ? (uint32_t)v : (uint32_t)(v >> 32);
            return (uint32_t)(((int32_t)(w << (31 - (J & 31)))) >> 31);
        } else {
            return (uint32_t)(((int32_t)(v << (31 - J))) >> 31);
        }
    }
    template <int J>
    __device__ __forceinline__ uint32_t low() const {
        return ext<J>(lt) | (ext<J>(eq) & pm);
    }
};

template <int J, int N, class Fn>
__device__ __forceinline__ void static_for(Fn &&f) {
    if constexpr (J < N) {
        f(std::integral_constant<int, J>{});
        static_for<J + 1, N>(f);
    }
}

// The base cases of Alg. 1 and Alg. 2 on canonical cells in LDS.
template <class F>
struct FermatOps : F {
    using F::C;
    using F::W;

    // v = sgn * (Lo - Hi) for x rotated left by t bits within N bits: Lo are the
    // bits that stay below 2^N, Hi the bits that wrapped (they count negatively).
    // Returns the borrow out of the element.
    // Limbs l C - qp + i (mod W), i = 0..C, of the element at x (the lane's
    // chunk shifted down by qp limbs).  For one element per wave they lie in
    // LDS rows row0 + i (column col0) and row0 + i - C (column col0 + 1), with
    // row0 the same for every lane: one select between two bases per limb.
    __device__ __forceinline__ void rot_words(const uint32_t *x, uint32_t qp, uint32_t (&src)[C + 1]) const {
        if constexpr (F::S == 64 && C > 1) {
            const uint32_t row0 = __builtin_amdgcn_readfirstlane((0u - qp) & (uint32_t)(C - 1));
            const uint32_t col0 = ((this->l * C - qp) & (uint32_t)(W - 1)) / C, col1 = (col0 + 1u) & 63u;
            const uint32_t oA = row0 * 64u + col0;
            const uint32_t oB = row0 * 64u + col1 - 64u * C;  // used only where oB + 64 i >= 0
#pragma unroll
            for (int i = 0; i <= C; ++i) src[i] = x[((uint32_t)i + row0 < (uint32_t)C ? oA : oB) + 64u * i];
        } else {
#pragma unroll
            for (int i = 0; i <= C; ++i) src[i] = x[F::addr((this->l * C - qp + (uint32_t)i) & (uint32_t)(W - 1))];
        }
    }

    template <bool NEG>
    __device__ __forceinline__ uint32_t rot_sub_impl(const uint32_t *x, const Rot<F> &rt, uint32_t (&v)[C]) const {
        uint32_t src[C + 1];
        rot_words(x, rt.qp, src);
        const RotMask<C> mk((int)rt.q - (int)(this->l * C), rt.pm);
        uint32_t b = 0;
        static_for<0, C>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const uint32_t r = __builtin_amdgcn_alignbit(src[j + 1], src[j], rt.c);
            const uint32_t low = mk.template low<j>();
            const uint32_t hp = r & low, lp = r & ~low;
            v[j] = NEG ? subb(hp, lp, b) : subb(lp, hp, b);
        });
        return this->settle(v, b, true);
    }
    __device__ __forceinline__ uint32_t rot_sub(const uint32_t *x, const Rot<F> &rt, uint32_t (&v)[C]) const {
        return rt.neg ? rot_sub_impl<true>(x, rt, v) : rot_sub_impl<false>(x, rt, v);
    }

    // x <- 2^e * (x + exc 2^N), x held raw in LDS; writes the canonical result and top
    __device__ __forceinline__ void twist_store(uint32_t *x, uint32_t *tp, uint32_t e, int exc) const {
        const Rot<F> rt(e);
        uint32_t v[C];
        const uint32_t bv = rot_sub(x, rt, v);
        // (x + exc 2^N) 2^e = v - bv 2^N + sg*exc*2^(N+t) = v - bv 2^N - sg*exc*2^t
        const uint32_t top = this->canon(v, -(int)bv, -rt.sg * exc, rt.t);
        this->st(x, v);
        if (this->l == 0u) *tp = top;
    }

    // TFT z=2 n=2: (x0, x1) <- (x0 + x1, 2^e (x0 - x1)), one pass over the limbs.
    // With R0, R1 the rotations of x0, x1 by t bits and Lo/Hi their bits that
    // stay below / wrap past 2^N: 2^t (x0 - x1) = (Lo0 - Hi0) - (Lo1 - Hi1)
    // = A - B with the disjoint merges A = Lo0 | Hi1, B = Lo1 | Hi0.
    template <bool NEG>
    __device__ __forceinline__ void t22_impl(uint32_t *x0, uint32_t *x1, uint32_t *tp0, uint32_t *tp1,
                                             const Rot<F> &rt) const {
        const int t0 = (int)*tp0, t1 = (int)*tp1;
        // twisted difference from the rotated words of both operands
        uint32_t d[C];
        uint32_t bd = 0;
        {
            uint32_t s0[C + 1], s1[C + 1];
            rot_words(x0, rt.qp, s0);
            rot_words(x1, rt.qp, s1);
            const RotMask<C> mk((int)rt.q - (int)(this->l * C), rt.pm);
            static_for<0, C>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                const uint32_t r0 = __builtin_amdgcn_alignbit(s0[j + 1], s0[j], rt.c);
                const uint32_t r1 = __builtin_amdgcn_alignbit(s1[j + 1], s1[j], rt.c);
                const uint32_t low = mk.template low<j>();
                const uint32_t A = (r1 & low) | (r0 & ~low);
                const uint32_t B = (r0 & low) | (r1 & ~low);
                d[j] = NEG ? subb(B, A, bd) : subb(A, B, bd);
            });
        }
        const uint32_t bv = this->settle(d, bd, true);
        __builtin_amdgcn_sched_barrier(0);  // keep the sum's loads after the difference (register pressure)
        // sum
        uint32_t a[C], b[C];
        this->ld(x0, a);
        this->ld(x1, b);
        uint32_t cy = 0;
#pragma unroll
        for (int j = 0; j < C; ++j) a[j] = addc(a[j], b[j], cy);
        const uint32_t ov = this->settle(a, cy, false);
        const uint32_t top0 = this->canon(a, (int)ov + t0 + t1, 0, 0u);
        const uint32_t top1 = this->canon(d, -(int)bv, rt.sg * (t1 - t0), rt.t);
        this->st(x0, a);
        this->st(x1, d);
        if (this->l == 0u) {
            *tp0 = top0;
            *tp1 = top1;
        }
    }
    __device__ void t22(uint32_t *x0, uint32_t *x1, uint32_t *tp0, uint32_t *tp1, uint32_t e) const {
        const Rot<F> rt(e);
        if (rt.neg)
            t22_impl<true>(x0, x1, tp0, tp1, rt);
        else
            t22_impl<false>(x0, x1, tp0, tp1, rt);
    }

    // TFT z=1 n=2: x1 <- 2^e x0
    __device__ void t21(const uint32_t *x0, uint32_t *x1, const uint32_t *tp0, uint32_t *tp1, uint32_t e) const {
        const Rot<F> rt(e);
        uint32_t v[C];
        const int t0 = (int)*tp0;
        const uint32_t bv = rot_sub(x0, rt, v);
        const uint32_t top = this->canon(v, -(int)bv, -rt.sg * t0, rt.t);
        this->st(x1, v);
        if (this->l == 0u) *tp1 = top;
    }

    // x0 <- x0 + x1
    __device__ void add2(uint32_t *x0, const uint32_t *x1, uint32_t *tp0, const uint32_t *tp1) const {
        uint32_t a[C], b[C], y[C];
        this->ld(x0, a);
        this->ld(x1, b);
        const int t0 = (int)*tp0, t1 = (int)*tp1;
        const uint32_t cy = this->add(y, a, b);
        const uint32_t top = this->canon(y, (int)cy + t0 + t1, 0, 0u);
        this->st(x0, y);
        if (this->l == 0u) *tp0 = top;
    }

    // x0 <- 2 x0 - x1 (x1 == nullptr: x0 <- 2 x0)
    __device__ void dbl_sub(uint32_t *x0, const uint32_t *x1, uint32_t *tp0, const uint32_t *tp1) const {
        uint32_t a[C], y[C];
        this->ld(x0, a);
        const int t0 = (int)*tp0;
        int exc;
        if (x1) {
            uint32_t b[C], d[C];
            this->ld(x1, b);
            const int t1 = (int)*tp1;
            const uint32_t bd = this->sub(d, a, b);
            const uint32_t cy = this->add(y, a, d);
            exc = (int)cy - (int)bd + 2 * t0 - t1;
        } else {
            const uint32_t cy = this->add(y, a, a);
            exc = (int)cy + 2 * t0;
        }
        const uint32_t top = this->canon(y, exc, 0, 0u);
        this->st(x0, y);
        if (this->l == 0u) *tp0 = top;
    }

    // ITFT n=2: (x0, x1) <- (x0 + 2^-e x1, x0 - 2^-e x1); einv = -e mod 2N
    __device__ void i2(uint32_t *x0, uint32_t *x1, uint32_t *tp0, uint32_t *tp1, uint32_t einv) const {
        const Rot<F> rt(einv);
        uint32_t y0[C], y1[C];
        const int t0 = (int)*tp0, t1 = (int)*tp1;
        const uint32_t bv = rot_sub(x1, rt, y1);  // 2^-e x1 = v - bv 2^N - sg t1 2^t, v held in y1
        this->ld(x0, y0);
        uint32_t c0 = 0, b1 = 0;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const uint32_t a = y0[j], v = y1[j];
            y0[j] = addc(a, v, c0);
            y1[j] = subb(a, v, b1);
        }
        c0 = this->settle(y0, c0, false);
        b1 = this->settle(y1, b1, true);
        const uint32_t top0 = this->canon(y0, (int)c0 + t0 - (int)bv, -rt.sg * t1, rt.t);
        const uint32_t top1 = this->canon(y1, -(int)b1 + t0 + (int)bv, rt.sg * t1, rt.t);
        this->st(x0, y0);
        this->st(x1, y1);
        if (this->l == 0u) {
            *tp0 = top0;
            *tp1 = top1;
        }
    }

    // ITFT n=1 f=1: (x0, x1) <- (2 x0 - x1, 2^e (x0 - x1)); z2 = false: x1 taken as 0
    __device__ void i1f1(uint32_t *x0, uint32_t *x1, uint32_t *tp0, uint32_t *tp1, uint32_t e, bool z2) const {
        uint32_t a[C], y[C];
        this->ld(x0, a);
        const int t0 = (int)*tp0;
        if (z2) {
            uint32_t b[C], d[C];
            this->ld(x1, b);
            const int t1 = (int)*tp1;
            const uint32_t bd = this->sub(d, a, b);
            const uint32_t cy = this->add(y, a, d);
            const uint32_t top0 = this->canon(y, (int)cy - (int)bd + 2 * t0 - t1, 0, 0u);
            this->st(x0, y);
            this->st(x1, d);
            if (this->l == 0u) *tp0 = top0;
            twist_store(x1, tp1, e, t0 - t1 - (int)bd);
        } else {
            t21(x0, x1, tp0, tp1, e);  // reads x0 before it changes
            const uint32_t cy = this->add(y, a, a);
            const uint32_t top0 = this->canon(y, (int)cy + 2 * t0, 0, 0u);
            this->st(x0, y);
            if (this->l == 0u) *tp0 = top0;
        }
    }

    // x0 <- 2^e x0 in place
    __device__ void scale(uint32_t *x0, uint32_t *tp0, uint32_t e) const {
        const int t0 = (int)*tp0;
        twist_store(x0, tp0, e, t0);
    }
};

}  // namespace tft
