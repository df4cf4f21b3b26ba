// Wave-level arithmetic of the persistent leaf executor in R = Z/(2^N+1):
// one element per wavefront, lane l holding limbs [l C, (l+1) C), W = 64 C,
// C = 4 .. 32; the base cases of Alg. 1 and Alg. 2 (L = 2) built from four
// primitives on cells in LDS.  Everything here is written against the wave
// primitives of wave_prims.hpp, so the same code also runs on the host under
// a lockstep emulation of one wavefront (tests/native).
#pragma once
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "desc.hpp"
#include "leaf2_addr.hpp"
#include "wave_prims.hpp"

namespace tft {
namespace lf2 {

template <int J, int N, class Fn>
TFT_DINL void static_for(Fn &&f) {
    if constexpr (J < N) {
        f(std::integral_constant<int, J>{});
        static_for<J + 1, N>(f);
    }
}

// Multiplication by 2^e, 0 <= e < 2N, as a rotation by t = e mod N bits with
// the bits that pass 2^N counted negatively (2^N = -1), and sign -1 if e >= N.
struct Rot {
    uint32_t t, q, qp, c, pm;
    bool neg;
    int sg;
    TFT_DINL Rot(uint32_t e, uint32_t N) {
        neg = e >= N;
        sg = neg ? -1 : 1;
        t = neg ? e - N : e;
        q = t >> 5;
        const uint32_t rb = t & 31u;
        pm = (1u << rb) - 1u;
        qp = q + (rb != 0u ? 1u : 0u);
        c = (32u - rb) & 31u;
    }
};

template <int C_>
struct Big {
    static constexpr int C = C_;
    static constexpr int W = 64 * C;
    static constexpr uint32_t N = 32u * W;
    static_assert(C >= 4 && C <= 32 && (C & (C - 1)) == 0, "four to 32 limbs per lane");

    uint32_t l;     // lane
    uint32_t zero;  // a zero the compiler cannot see through: keeps x + 0 + carry a carry chain

    TFT_DINL Big() : l(lane_id()), zero(opaque_zero()) {}

    TFT_DINL void ld(const uint32_t *sm, uint32_t e, uint32_t (&v)[C]) const {
        const uint32_t *p = sm + e + l;
#pragma unroll
        for (int j = 0; j < C; ++j) v[j] = p[64 * j];
    }
    TFT_DINL void st(uint32_t *sm, uint32_t e, const uint32_t (&v)[C]) const {
        uint32_t *p = sm + e + l;
#pragma unroll
        for (int j = 0; j < C; ++j) p[64 * j] = v[j];
    }

    // ---- rare cases, in LDS, one lane, rolled loops ----

    // Adds (SUB: subtracts) m at limb k0 of the element at e and carries
    // upward; returns the carry (borrow) out of limb W-1.  Wave-uniform: every
    // lane reads the same words, lane 0 writes.
    TFT_DINL uint32_t lds_ripple(uint32_t *sm, uint32_t e, uint32_t k0, uint32_t m, bool sub) const {
        uint32_t c = m;
#pragma unroll 1
        for (uint32_t k = k0; k < (uint32_t)W && c != 0u; ++k) {
            wave_sync();
            const uint32_t a = e + limb_pos(C, k);
            const uint32_t w = uni(sm[a]);
            const uint32_t r = sub ? w - c : w + c;
            const uint32_t nc = sub ? (w < c ? 1u : 0u) : (r < w ? 1u : 0u);
            if (l == 0u) sm[a] = r;
            c = nc;
        }
        return c;
    }

    // The stored element at e is V; its value is V + X 2^N + corr 2^cbit plus
    // +1 (SUB: -1) at limb l C for every lane l in pend.  Makes it canonical
    // in place and writes its top word.
    TFT_DINL void lds_finish(uint32_t *sm, uint32_t e, uint32_t ti, uint64_t pend, bool sub, int X, int corr,
                             uint32_t cbit) const {
#pragma unroll 1
        while (pend != 0ull) {
            const uint32_t lp = (uint32_t)__builtin_ctzll(pend);
            pend &= pend - 1ull;
            (void)lds_ripple(sm, e, lp * (uint32_t)C, 1u, sub);  // stops inside the chunk
        }
        if (corr != 0) {
            const bool cs = corr < 0;
            const uint64_t m64 = (uint64_t)(uint32_t)(cs ? -corr : corr) << (cbit & 31u);
            const uint32_t k0 = cbit >> 5;
            int o = (int)lds_ripple(sm, e, k0, (uint32_t)m64, cs);
            const uint32_t hi = (uint32_t)(m64 >> 32);
            if (hi != 0u) o += (k0 + 1u < (uint32_t)W) ? (int)lds_ripple(sm, e, k0 + 1u, hi, cs) : (int)hi;
            X += cs ? -o : o;
        }
        // value = V + X 2^N = V - X (mod 2^N + 1)
        int X1 = 0;
        if (X > 0) X1 = lds_ripple(sm, e, 0u, (uint32_t)X, true) ? -1 : 0;       // borrow: value = V' + 1
        else if (X < 0) X1 = lds_ripple(sm, e, 0u, (uint32_t)(-X), false) ? 1 : 0;  // carry: value = V' - 1
        uint32_t top = 0u;
        if (X1 < 0) {
            if (lds_ripple(sm, e, 0u, 1u, false)) top = 1u;  // V' was 2^N - 1: the limbs are now zero
        } else if (X1 > 0) {
            if (lds_ripple(sm, e, 0u, 1u, true)) {  // V' was 0: the value is -1 = 2^N
                uint32_t z[C];
#pragma unroll
                for (int j = 0; j < C; ++j) z[j] = 0u;
                wave_sync();  // after lane 0's last ripple store to these words
                st(sm, e, z);
                top = 1u;
            }
        }
        if (l == 0u) sm[ti] = top;
    }

    // ---- the common path, in registers ----

    // Carry lookahead over the 64 lanes: G = lanes emitting a carry (borrow)
    // into the next lane, P = lanes whose chunk passes an incoming carry on
    // (all ones; SUB: all zeros).  Returns the carries into the lanes,
    // ((G | P) + G) ^ P, and in *out the carry out of lane 63.
    template <bool SUB>
    TFT_DINL uint64_t lookahead(const uint32_t (&v)[C], uint64_t G, uint32_t *out) const {
        uint32_t acc = v[0];
#pragma unroll
        for (int j = 1; j < C; ++j) acc = SUB ? (acc | v[j]) : (acc & v[j]);
        const uint64_t P = ballot(SUB ? acc == 0u : acc == ~0u);
        const uint64_t X = G | P;
        const uint64_t cin = (X + G) ^ P;
        *out = (uint32_t)(((G >> 63) | ((P >> 63) & (cin >> 63))) & 1ull);
        return cin;
    }

    // v += 1 (SUB: -= 1) at limb 0 of the lanes in m, carried through the
    // whole chunk (the carry out of a chunk is accounted for by the caller).
    template <bool SUB>
    TFT_DINL void lane_ripple(uint32_t (&v)[C], uint64_t m) const {
        const uint32_t one = lane_bit(m) ? 1u : 0u;
        uint32_t c = 0;
        v[0] = SUB ? subb(v[0], one, c) : addc(v[0], one, c);
#pragma unroll
        for (int j = 1; j < C; ++j) v[j] = SUB ? subb(v[j], zero, c) : addc(v[j], zero, c);
        // the last carry is dropped: keep the next chain from absorbing these limbs
#pragma unroll
        for (int j = 0; j < C; ++j) opaque(v[j]);
    }

    // Slow path of finish (long carry runs, or an excess that limb 0 of lane
    // 0 cannot absorb): straight-line register code that ends with the store,
    // so the common path never merges with it.
    template <bool SUB>
    TFT_DINL void finish_slow(uint32_t *sm, uint32_t (&v)[C], uint64_t G, int exc, int corr, uint32_t cbit,
                              uint32_t e, uint32_t ti) const {
        // carries between lanes
        uint32_t ovf;
        const uint64_t cin = lookahead<SUB>(v, G, &ovf);
        lane_ripple<SUB>(v, cin);
        // value = v + X 2^N (+ corr 2^cbit) = v - X: add m = -X at bit 0 as
        // one addition of A = m mod 2^N (A = 2^N + m for m < 0), whose limbs
        // are all ones except limb 0 when m < 0
        const int X = exc + (SUB ? -(int)ovf : (int)ovf);
        const int m = -X;
        const uint32_t fillA = m < 0 ? ~0u : 0u;
        uint32_t c = 0;
        v[0] = addc(v[0], l == 0u ? (uint32_t)m : fillA, c);
#pragma unroll
        for (int j = 1; j < C; ++j) v[j] = addc(v[j], fillA, c);
        uint32_t o2;
        const uint64_t cin2 = lookahead<false>(v, ballot(c != 0u), &o2);
        lane_ripple<false>(v, cin2);
        // v + m = v' + (o2 - [m < 0]) 2^N
        const int o = (int)o2 - (m < 0 ? 1 : 0);
        // value = v' + o 2^N = v' - o, |o| <= 1: limb 0 of lane 0 only
        const uint32_t y0 = readlane(v[0], 0);
        uint32_t top = 0u;
        bool zero = false;
        if (o > 0) {  // v' < |m|
            if (y0 == 0u)
                top = 1u;  // -1 = 2^N
            else if (l == 0u)
                v[0] = y0 - 1u;
        } else if (o < 0) {  // v' >= 2^N - |m|: every limb but limb 0 is all ones
            if (y0 == 0xFFFFFFFFu) {
                top = 1u;  // 2^N: the limbs become zero
                zero = true;
            } else if (l == 0u) {
                v[0] = y0 + 1u;
            }
        }
        st(sm, e, v);
        if (zero) {  // written over the store: no second version of v in registers
            uint32_t *p = sm + e + l;
#pragma unroll
            for (int j = 0; j < C; ++j) p[64 * j] = 0u;
        }
        if (corr != 0)
            lds_finish(sm, e, ti, 0ull, SUB, (int)top, corr, cbit);  // a top word was involved: rare
        else if (l == 0u)
            sm[ti] = top;
    }

    // v holds the per-lane chunks of a limb chain (SUB: a difference) whose
    // carry (borrow) out of each chunk is co; the value is v + exc 2^N +
    // corr 2^cbit.  Moves the carries between lanes, makes the value
    // canonical and stores it at e with its top word at ti.  Common path:
    // every carry into a lane stops at its limb 0 and limb 0 of lane 0
    // absorbs the excess (a few instructions); otherwise finish_slow.
    template <bool SUB>
    TFT_DINL void finish(uint32_t *sm, uint32_t (&v)[C], uint32_t co, int exc, int corr, uint32_t cbit, uint32_t e,
                         uint32_t ti) const {
        const uint64_t G = ballot(co != 0u);
        const uint64_t cin = G << 1;
        const uint64_t pass0 = ballot(SUB ? v[0] == 0u : v[0] == ~0u);
        const int X = exc + (SUB ? -(int)(G >> 63) : (int)(G >> 63));
        const uint32_t y0 = readlane(v[0], 0);  // lane 0 takes no carry from below
        const bool absorb = X == 0 || (X > 0 ? (y0 >= (uint32_t)X) : (y0 <= 0xFFFFFFFFu - (uint32_t)(-X)));
        if ((cin & pass0) == 0ull && corr == 0 && absorb) {
            const uint32_t c = lane_bit(cin) ? 1u : 0u;
            v[0] = SUB ? v[0] - c : v[0] + c;
            if (l == 0u) v[0] = y0 - (uint32_t)X;
            st(sm, e, v);
            if (l == 0u) sm[ti] = 0u;
            return;
        }
        finish_slow<SUB>(sm, v, G, exc, corr, cbit, e, ti);
    }

    // Words of the element at cell offset e rotated down by qp limbs:
    // src[i] = limb (l C - qp + i) mod W, i = 0..C.
    TFT_DINL void rot_words(const uint32_t *sm, uint32_t e, uint32_t qp, uint32_t (&src)[C + 1]) const {
        const uint32_t sA = uni((uint32_t)C - rot_row0(C, qp));  // words [0, sA) come from base A
        // LDS byte addresses of the two bases, selected per word (the word's
        // own offset is the load's immediate); e >= W keeps base B inside the
        // allocation
        uint32_t bA = lds_addr(sm) + 4u * rot_base_a(C, e, l, qp), bB = lds_addr(sm) + 4u * rot_base_b(C, e, l, qp);
        opaque(bA);
        opaque(bB);
#pragma unroll
        for (int i = 0; i <= C; ++i) src[i] = lds_word(sm, ((uint32_t)i < sA ? bA : bB) + 256u * (uint32_t)i);
    }

    // dst <- 2^e (x + t 2^N), x the element at src with top t (a canonical
    // residue): the rotation of x by t bits gives Lo - Hi (sign -1 if e >= N),
    // Lo the bits that stay below 2^N, Hi the bits that wrapped.
    template <bool NEG>
    TFT_DINL void twist_impl(uint32_t *sm, uint32_t es, uint32_t ed, uint32_t ti, int top, const Rot &rt) const {
        uint32_t v[C];
        uint32_t b = 0;
        {
            uint32_t src[C + 1];
            rot_words(sm, es, rt.qp, src);
            wave_sync();  // every lane has read before any lane stores (es may be ed)
            // The wrapped part of limb j of lane l is r & M_j: M_j is all ones
            // below the split limb q = qa C + jq, pm at it, zero above.  Lanes
            // below qa wrap whole, lanes above not at all; lane qa takes M_j
            // from lane j of a per-lane table, read as a wave-uniform value.
            const uint32_t qa = rt.q / (uint32_t)C, jq = rt.q % (uint32_t)C;
            uint32_t fv = l < qa ? ~0u : 0u, am = l == qa ? ~0u : 0u;
            opaque(fv);  // plain words to the compiler: one and-or per limb, not a select
            opaque(am);
            const uint32_t stab = l < jq ? ~0u : (l == jq ? rt.pm : 0u);
            static_for<0, C>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                const uint32_t r = alignbit(src[j + 1], src[j], rt.c);
                uint32_t M = (am & readlane(stab, j)) | fv;  // one and-or, no select
                opaque(M);                                    // formed once, used twice
                // Lo - Hi with Lo = r & ~M, Hi = r & M: (r ^ M) - M, since
                // r ^ M = Lo + (M - Hi); the negated form is M - (r ^ M)
                const uint32_t x = r ^ M;
                v[j] = NEG ? subb(M, x, b) : subb(x, M, b);
                // groups of 8 limbs: the scheduler may not hoist every limb's
                // shifts and masks ahead of the borrow chain (register pressure)
                if constexpr ((j & 7) == 7) sched_barrier();
            });
        }
        // 2^e (x + t 2^N) = v - bv 2^N - sg t 2^t
        finish<true>(sm, v, b, 0, -rt.sg * top, rt.t, ed, ti);
    }
    TFT_DINL void twist(uint32_t *sm, uint32_t es, uint32_t ed, uint32_t ti, int top, uint32_t ex) const {
        const Rot rt(ex, N);
        if (rt.neg)
            twist_impl<true>(sm, es, ed, ti, top, rt);
        else
            twist_impl<false>(sm, es, ed, ti, top, rt);
    }

    // sum and difference chains of two loaded elements
    TFT_DINL uint32_t chain_add(uint32_t (&r)[C], const uint32_t (&a)[C], const uint32_t (&b)[C]) const {
        uint32_t c = 0;
#pragma unroll
        for (int j = 0; j < C; ++j) r[j] = addc(a[j], b[j], c);
        return c;
    }
    TFT_DINL uint32_t chain_sub(uint32_t (&r)[C], const uint32_t (&a)[C], const uint32_t (&b)[C]) const {
        uint32_t c = 0;
#pragma unroll
        for (int j = 0; j < C; ++j) r[j] = subb(a[j], b[j], c);
        return c;
    }

    // ---- the four primitives every base case is made of ----

    // (xi, xj) <- (xi + xj, xi - xj): the difference goes canonical into xj,
    // then the sum into xi (a scheduling barrier keeps the two limb chains
    // apart: at most three element vectors live)
    TFT_DINL void p_addsub(uint32_t *sm, uint32_t ei, uint32_t ej, uint32_t ii, uint32_t ij) const {
        wave_sync();
        const int ti = (int)uni(sm[ii]), tj = (int)uni(sm[ij]);
        uint32_t a[C], b[C];
        ld(sm, ei, a);
        ld(sm, ej, b);
        // the sum and difference chains interleaved limb by limb, in place: two
        // independent carries, so neither chain waits on its own carry
        uint32_t cy = 0, bd = 0;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const uint32_t t = a[j];
            a[j] = addc(t, b[j], cy);
            b[j] = subb(t, b[j], bd);
        }
        finish<true>(sm, b, bd, ti - tj, 0, 0u, ej, ij);
        sched_barrier();
        finish<false>(sm, a, cy, ti + tj, 0, 0u, ei, ii);
    }
    // xi <- xi + xj (i = j doubles)
    TFT_DINL void p_add(uint32_t *sm, uint32_t ei, uint32_t ej, uint32_t ii, uint32_t ij) const {
        wave_sync();
        const int ti = (int)uni(sm[ii]), tj = (int)uni(sm[ij]);
        uint32_t a[C], b[C];
        ld(sm, ei, a);
        ld(sm, ej, b);
        const uint32_t cy = chain_add(a, a, b);
        finish<false>(sm, a, cy, ti + tj, 0, 0u, ei, ii);
    }
    // xj <- xi - xj
    TFT_DINL void p_subr(uint32_t *sm, uint32_t ei, uint32_t ej, uint32_t ii, uint32_t ij) const {
        wave_sync();
        const int ti = (int)uni(sm[ii]), tj = (int)uni(sm[ij]);
        uint32_t a[C], b[C];
        ld(sm, ei, a);
        ld(sm, ej, b);
        const uint32_t bd = chain_sub(b, a, b);
        finish<true>(sm, b, bd, ti - tj, 0, 0u, ej, ij);
    }
    // xj <- 2^e xi
    TFT_DINL void p_twist(uint32_t *sm, uint32_t ei, uint32_t ej, uint32_t ii, uint32_t ij, uint32_t ex) const {
        wave_sync();
        twist(sm, ei, ej, ij, (int)uni(sm[ii]), ex);
    }
};

// Base cases of Alg. 1 and Alg. 2 (L = 2) as sequences of the primitives,
// packed 8 bits per step (first step in the low byte): kind (bits 0-1:
// 1 addsub, 2 add, 3 reverse subtract; 0 with bit 4: twist), operand i
// (bit 2), operand j (bit 3), twist exponent (bits 5-6: 0 e, 1 -e, 2 the
// inverse of 2).
enum : uint32_t { M_ADDSUB = 1, M_ADD = 2, M_SUBR = 3, M_TWIST = 16 };
constexpr uint32_t mop(uint32_t kind, uint32_t i, uint32_t j, uint32_t em = 0) {
    return kind | (i << 2) | (j << 3) | (em << 5);
}
TFT_DINL uint32_t base_case_steps(uint32_t code) {
    switch (code) {
        case OP_T22:  // (x0 + x1, zeta (x0 - x1))
            return mop(M_ADDSUB, 0, 1) | mop(M_TWIST, 1, 1) << 8;
        case OP_T21:  // x1 = zeta x0
            return mop(M_TWIST, 0, 1);
        case OP_T12:  // x0 = x0 + x1
            return mop(M_ADD, 0, 1);
        case OP_I2:  // x1 = x1 / zeta, then (x0 + x1, x0 - x1)
            return mop(M_TWIST, 1, 1, 1) | mop(M_ADDSUB, 0, 1) << 8;
        case OP_I1F1Z2:  // x1 = x0 - x1, x0 = x0 + x1 (= 2 x0 - x1), x1 = zeta x1
            return mop(M_SUBR, 0, 1) | mop(M_ADD, 0, 1) << 8 | mop(M_TWIST, 1, 1) << 16;
        case OP_I1F1Z1:  // x1 = zeta x0, x0 = 2 x0
            return mop(M_TWIST, 0, 1) | mop(M_ADD, 0, 0) << 8;
        case OP_I1F0Z2:  // x1 = x0 - x1 (not an output), x0 = x0 + x1 = 2 x0 - x1
            return mop(M_SUBR, 0, 1) | mop(M_ADD, 0, 1) << 8;
        case OP_I1F0Z1:  // x0 = 2 x0
            return mop(M_ADD, 0, 0);
        case OP_I0Z2:  // x0 = (x0 + x1) / 2
            return mop(M_ADD, 0, 1) | mop(M_TWIST, 0, 0, 2) << 8;
        case OP_I0Z1:  // x0 = x0 / 2
            return mop(M_TWIST, 0, 0, 2);
        default: return 0u;
    }
}

// One base case (opcode, cells i0 and i1, exponent (s 2^alog + b) mod 2N of
// the job's twist s) on the leaf in LDS, run by one wave; the job's cells start
// at LDS cell cofs.
template <int C>
TFT_DINL void base_case(const Big<C> &ar, uint32_t *sm, const LeafOp &o, uint32_t s, uint32_t ord_mask,
                        uint32_t cofs = 0u) {
    constexpr uint32_t W = Big<C>::W;
    const uint32_t i01[2] = {((o.w0 >> 4) & 16383u) + cofs, ((o.w0 >> 18) & 16383u) + cofs};
    const uint32_t ex = (uint32_t)((((uint64_t)s << op_alog(o)) + (uint64_t)op_b(o)) & ord_mask);
    const uint32_t exs[3] = {ex, (0u - ex) & ord_mask, ord_mask};  // e, -e, 2N - 1 (2^(2N-1) = 1/2)
    for (uint32_t seq = base_case_steps(o.w0 & 15u); seq != 0u; seq >>= 8) {
        const uint32_t m = seq & 255u;
        const uint32_t ii = i01[(m >> 2) & 1u], ij = i01[(m >> 3) & 1u];
        const uint32_t ei = cell_base(W, ii), ej = cell_base(W, ij);
        switch (m & 19u) {
            case M_ADDSUB: ar.p_addsub(sm, ei, ej, ii, ij); break;
            case M_ADD: ar.p_add(sm, ei, ej, ii, ij); break;
            case M_SUBR: ar.p_subr(sm, ei, ej, ii, ij); break;
            case M_TWIST: ar.p_twist(sm, ei, ej, ii, ij, exs[(m >> 5) & 3u]); break;
            default: break;
        }
    }
}

}  // namespace lf2
}  // namespace tft
