// Pointwise products in R = Z/(2^N+1) for large N by one more level of
// Schoenhage-Strassen (the recursion the SS product is built on, Sect. 5.1):
// a product a b mod 2^N+1 is a negacyclic convolution of K pieces of P = N/K
// bits (x = 2^P, x^K = 2^N = -1), computed with length-K transforms over the
// inner ring Z/(2^N'+1).
//
//   pieces   a = sum_i a_i 2^(P i), 0 <= a_i < 2^P, i < K
//   twist    A_i = a_i psi^i, psi = 2^(N'/K) of order 2K, so that the cyclic
//            convolution of the A_i is the negacyclic one of the a_i
//   forward  radix-2 decimation in frequency, omega = 2^(2N'/K)
//   products C_j = A_j B_j mod 2^N'+1 (bit-reversed positions j)
//   inverse  radix-2 decimation in time with omega^-1 (gives K times the
//            cyclic convolution, in natural order)
//   untwist  c_i = (K psi^i)^-1 V_i, read as a signed integer: |c_i| < K 2^(2P)
//            and N' >= 2P + log2 K + 2, so it is exact
//   recombine a b = sum_i c_i 2^(P i) mod 2^N+1: per limb j, the sums of the
//            positive and of the negative words landing there (at most three
//            pieces overlap a limb; wrapped words change sign)
//
// N' = 32 WI is a multiple of 16 K, so every twiddle of the transforms is a
// shift by whole 32-bit limbs; only the twist and untwist shift by bits.
//
// The transforms work on signed digits: a cell is WI int64 digits x_d with
// value sum_d x_d 2^(32 d) (mod 2^N'+1), carries left in the digits.  A sum
// or difference is digit by digit, and a product by 2^(32 q) moves digit d to
// d + q, negated where it passes 2^N' = -1: no carry chains, so a lane takes a
// digit of a butterfly and all lanes work on every level.  Digits start below
// 2^32 in magnitude and each level adds one bit, so six levels stay far inside
// 64 bits.  A cell's carries are resolved (serially, a lane a cell) only before
// the inner products and before the untwist, into a normalised cell: WI limbs
// and a word h in {0, 1} with value L + h 2^N' (h = 1 only for 2^N').
//
// The functions below are for one lane; a kernel spreads digits, cells and
// product columns over lanes and separates the phases with barriers.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define TFT_NEST_HD __host__ __device__ __forceinline__
#else
#define TFT_NEST_HD inline
#endif

namespace tft {
namespace nest {

template <int W>
struct Cfg;
// N = 16384: 64 pieces of 256 bits over Z/(2^1024+1) (omega = 2^32, psi = 2^16)
template <>
struct Cfg<512> {
    static constexpr int K = 64, WI = 32;
};
// N = 32768: 64 pieces of 512 bits over Z/(2^2048+1) (omega = 2^64, psi = 2^32)
template <>
struct Cfg<1024> {
    static constexpr int K = 64, WI = 64;
};
// N = 65536: 64 pieces of 1024 bits over Z/(2^3072+1) (omega = 2^96, psi = 2^48)
template <>
struct Cfg<2048> {
    static constexpr int K = 64, WI = 96;
};
// N = 131072: 64 pieces of 2048 bits over Z/(2^5120+1) (omega = 2^160, psi = 2^80)
template <>
struct Cfg<4096> {
    static constexpr int K = 64, WI = 160;
};

template <int W_>
struct Nest {
    static constexpr int W = W_;
    static constexpr int K = Cfg<W>::K;
    static constexpr int LOGK = K == 64 ? 6 : -1;
    static constexpr int WI = Cfg<W>::WI;      // inner limbs
    static constexpr int WP = WI + 1;          // cell pitch in LDS words (limbs, then h)
    static constexpr int PL = W / K;           // limbs of a piece
    static constexpr int NR = 2 * PL + 1;      // limbs of |c_i| < 2^(2P + log2 K)
    static constexpr int G = 4;                // column groups (waves) of the inner products
    static constexpr int NC = WI / G;          // product columns of one wave
    static constexpr uint32_t NI = 32u * WI;   // N'
    static constexpr int LB = 8;               // limbs a serial loop loads before it computes
    static_assert(LOGK > 0 && W % K == 0, "pieces");
    static_assert((2 * WI) % K == 0, "omega is a shift by whole limbs");
    static_assert(32 * WI >= 64 * PL + LOGK + 2, "N' holds the signed coefficients");
    static_assert(NC % 4 == 0 && NC * G == WI, "columns come in groups of four");
    static_assert(WI % LB == 0 && WI % 4 == 0, "limb blocks");

    // LDS words (offsets), sized so that two workgroups share a compute
    // unit: one region of K digit cells (pitch DP words = WI + 1 int64), the
    // normalised cells of a (pitch WP), and the column carries.  a is
    // transformed and normalised first; then b goes through the digit region
    // and is normalised in place there (a cell's limb m lands on words its
    // digits have already left); the products overwrite a's normalised
    // cells; the inverse and the untwist use the digit region again; |c_i|
    // and signs overwrite the normalised cells in place; the recombination's
    // four limb arrays take [0, 4W) of the digit region.
    static constexpr int DP = 2 * WI + 2;
    static constexpr int D = 0, LA = K * DP, CW = LA + K * WP;
    static constexpr int WORDS = CW + 2 * G * K;
    static constexpr int PA = 0, PB = W, P0 = 2 * W, N0 = 3 * W;  // recombination arrays
    static_assert(4 * W <= K * DP, "recombination arrays in the digit region");
    static_assert(NR + 1 <= WP, "|c_i| in place of the normalised cell");

    TFT_NEST_HD static int32_t geth(const uint32_t *c) { return (int32_t)c[WI]; }
    TFT_NEST_HD static void seth(uint32_t *c, int64_t h) { c[WI] = (uint32_t)(int32_t)h; }

    // (L, h) -> the residue in [0, 2^N'] (h becomes 0, or 1 with L = 0 for
    // 2^N'); h is passed in, as it may exceed the cell's h word
    TFT_NEST_HD static void normalize(uint32_t *c, int64_t h) {
        int64_t carry = -h;  // L - h
        for (int m = 0; m < WI && carry != 0; ++m) {
            const int64_t acc = (int64_t)c[m] + carry;
            c[m] = (uint32_t)acc;
            carry = acc >> 32;
        }
        // value = L' + carry 2^N' = L' - carry, carry in {-1, 0, 1}
        int64_t c2 = -carry;
        for (int m = 0; m < WI && c2 != 0; ++m) {
            const int64_t acc = (int64_t)c[m] + c2;
            c[m] = (uint32_t)acc;
            c2 = acc >> 32;
        }
        if (c2 < 0) {  // L' was 0 and the value is -1: the residue 2^N'
            for (int m = 0; m < WI; ++m) c[m] = 0u;
            seth(c, 1);
        } else {
            seth(c, c2);  // 1: L' + 1 reached 2^N' (limbs already 0)
        }
    }
    TFT_NEST_HD static void normalize(uint32_t *c) { normalize(c, geth(c)); }

    // The split of cell i (piece i, limbs limb(i PL ..), times psi^i = 2^t,
    // t = i N'/K bits = 32 Q + r): limb s of piece * 2^r, s = 0 .. PL, moves
    // to digit s + Q, negated past 2^N'; every other digit is 0.  Piece
    // limbs k0 .. k1-1 (and, for k1 = PL, the top limb s = PL) are written by
    // split_part, so that lanes of one wave can take cells and waves ranges
    // of k; split_zero writes the zero digits d in [d0, d1).
    TFT_NEST_HD static void twist_of(int i, int &Q, uint32_t &r) {
        const uint32_t t = (uint32_t)i * (NI / K);
        Q = (int)(t >> 5);
        r = t & 31u;
    }
    template <class Limb>
    // Piece limbs [k0, k1) of cell i, k1 - k0 = PL / G: all the limbs they
    // need (and limb k0 - 1) are read first, in a loop of fixed length, so
    // that the reads are in flight together instead of one after another.
    TFT_NEST_HD static void split_part(Limb limb, int i, int k0, int k1, int64_t *cell) {
        constexpr int KP = PL / G;
        int Q;
        uint32_t r;
        twist_of(i, Q, r);
        uint32_t w[KP + 1];  // w[t] = limb k0 + t - 1 of the piece (0 below limb 0)
#pragma unroll
        for (int t = 0; t <= KP; ++t) {
            const int s = k0 + t - 1;
            const uint32_t x = limb(i * PL + (s > 0 ? s : 0));
            w[t] = s >= 0 ? x : 0u;
        }
        auto put = [&](int s, uint32_t cur, uint32_t prev) {
            const uint32_t v = (cur << r) | (r ? prev >> (32u - r) : 0u);
            int d = s + Q;
            const bool neg = d >= WI;
            if (neg) d -= WI;
            cell[d] = neg ? -(int64_t)v : (int64_t)v;
        };
#pragma unroll
        for (int t = 1; t <= KP; ++t) put(k0 + t - 1, w[t], w[t - 1]);
        if (k1 == PL) put(PL, 0u, w[KP]);  // the bits of the top limb shifted past the piece
    }
    TFT_NEST_HD static void split_zero(int i, int d0, int d1, int64_t *cell) {
        int Q;
        uint32_t r;
        twist_of(i, Q, r);
        for (int d = d0; d < d1; ++d) {
            int s = d - Q;
            if (s < 0) s += WI;
            if (s > PL) cell[d] = 0;
        }
    }

    // twiddle exponent (limbs) of butterfly offset off at half-size hs:
    // w^off = 2^(off N'/hs) = 2^(32 q)
    TFT_NEST_HD static int twiddle_limbs(int off, int hs) { return off * (WI / hs); }

    // resolve the carries of a digit cell into a normalised cell; out may be
    // the digit cell itself (limb m is written after digits up to m have
    // been read, a block of LB at a time)
    TFT_NEST_HD static void norm_digits(const int64_t *D, uint32_t *out) {
        int64_t c = 0;
        for (int m0 = 0; m0 < WI; m0 += LB) {
            int64_t v[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) v[u] = D[m0 + u];
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int64_t acc = v[u] + c;
                out[m0 + u] = (uint32_t)acc;
                c = acc >> 32;
            }
        }
        normalize(out, c);
    }

    // digit d of V_i 2^(-log2 K - i N'/K) (mod 2^N'+1) for the normalised
    // inverse-transform output V_i: the untwist and the 1/K of the inverse.
    // The factor is 2^s, s = 32 Q + r (a Q past WI takes the sign of 2^N');
    // U = V 2^r has limbs u_m = V[m] << r | V[m-1] >> (32 - r) and a part
    // u_top 2^N' = -u_top, which lands on digit Q.
    TFT_NEST_HD static int64_t untwist_digit(const uint32_t *V, int i, int d) {
        const uint32_t s = (2u * NI - (uint32_t)LOGK - (uint32_t)i * (NI / K)) % (2u * NI);
        int Q = (int)(s >> 5);
        const uint32_t r = s & 31u;
        int sigma = 1;
        if (Q >= WI) {
            Q -= WI;
            sigma = -1;
        }
        int m = d - Q, sg = sigma;
        if (m < 0) {
            m += WI;
            sg = -sg;
        }
        const uint32_t u = (V[m] << r) | ((m > 0 && r) ? V[m - 1] >> (32u - r) : 0u);
        int64_t val = sg < 0 ? -(int64_t)u : (int64_t)u;
        if (d == Q) {
            const int64_t utop = (int64_t)((r ? V[WI - 1] >> (32u - r) : 0u) + (V[WI] << r));
            val -= sigma < 0 ? -utop : utop;
        }
        return val;
    }

    // the signed coefficient held by a normalised cell (|c| < 2^(2P + log2 K)):
    // magnitude limbs [0, NR) and sign (1 = negative) at mg[NR].  Above
    // 2^(N'-1) the residue stands for V - (2^N' + 1).
    TFT_NEST_HD static void magnitude(const uint32_t *work, uint32_t *mg) {
        const bool neg = geth(work) != 0 || (work[WI - 1] >> 31) != 0u;
        if (neg) {
            // 2^N' + 1 - V = ~V + 2 for V < 2^N'; 1 for V = 2^N'
            if (geth(work) != 0) {
                for (int m = 0; m < NR; ++m) mg[m] = m == 0 ? 1u : 0u;
            } else {
                uint64_t c = 2;
                for (int m0 = 0; m0 < NR; m0 += 4) {
                    uint32_t v[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) v[u] = m0 + u < NR ? work[m0 + u] : 0u;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const uint64_t t = (uint64_t)(uint32_t)~v[u] + c;
                        v[u] = (uint32_t)t;
                        c = t >> 32;
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (m0 + u < NR) mg[m0 + u] = v[u];
                }
            }
        } else {
            for (int m = 0; m < NR; ++m) mg[m] = work[m];
        }
        mg[NR] = neg ? 1u : 0u;
    }

    // the product of two normalised cells when either is 2^N' (= -1): written
    // to out (which may be a or b)
    TFT_NEST_HD static void special_product(const uint32_t *a, const uint32_t *b, uint32_t *out) {
        const bool ta = geth(a) != 0, tb = geth(b) != 0;
        if (ta && tb) {  // (-1)(-1) = 1
            for (int m = 0; m < WI; ++m) out[m] = m == 0 ? 1u : 0u;
            seth(out, 0);
            return;
        }
        // -v = 2^N' + 1 - v = ~v + 2 (an integer up to 2^N' + 1; its carry out
        // of the limbs becomes h)
        const uint32_t *v = ta ? b : a;
        uint64_t c = 2;
        for (int m = 0; m < WI; ++m) {
            const uint64_t s = (uint64_t)(uint32_t)~v[m] + c;
            out[m] = (uint32_t)s;
            c = s >> 32;
        }
        seth(out, (int64_t)c);
        normalize(out);
    }

    // limb j of the result: positive and negative word sums from the pieces
    // that overlap it (pieces past 2^N wrap around with the opposite sign)
    TFT_NEST_HD static void gather(const uint32_t *mgs, int j, uint64_t &pos, uint64_t &neg) {
        constexpr int MGP = WP;  // |c_i| sits in place of normalised cell i
        pos = 0;
        neg = 0;
        const int it = j / PL;
        for (int d = 0; d < 3; ++d) {
            int i = it - d;
            const bool wrapped = i < 0;
            if (wrapped) i += K;
            const int m = j + (wrapped ? W : 0) - i * PL;
            if (m < NR) {
                const uint32_t *mg = mgs + i * MGP;
                if ((mg[NR] != 0u) != wrapped)
                    neg += mg[m];
                else
                    pos += mg[m];
            }
        }
    }

    // the column part of one inner product: columns k0 .. k0 + NC - 1 of
    // C = A B mod 2^N'+1 for normalised cells A, B with h = 0.  With
    // A2 = [A, ~A] and T_k = sum_{j>k} B_j, column k is
    //   d_k = S_k + T_k - 2^32 T_k,  S_k = sum_j B_j A2[(k - j) mod 2 WI]
    // (the negacyclic wrap without sign tests).  out gets the NC limbs of
    // sum_k d_k 2^(32 (k - k0)) and the return value its carry into limb
    // k0 + NC (signed).  mac(acc, cy, aw, bj) adds aw[c] bj into the 64-bit
    // acc[c] and counts its wraps in cy[c].
    template <class Mac>
    TFT_NEST_HD static int64_t columns(const uint32_t *A, const uint32_t *B, int k0, uint32_t (&out)[NC], Mac mac) {
        uint64_t acc[NC];
        uint32_t cy[NC], aw[NC];
        for (int c = 0; c < NC; ++c) {
            acc[c] = 0;
            cy[c] = 0;
            aw[c] = A[k0 + c];
        }
        for (int j0 = 0; j0 < WI; j0 += 4) {
            // the next four B limbs and window entries, loaded together
            uint32_t bj[4], an[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                bj[u] = B[j0 + u];
                int t = k0 - j0 - u - 1;
                if (t < 0) t += 2 * WI;
                an[u] = t < WI ? A[t] : ~A[t - WI];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                mac(acc, cy, aw, bj[u]);
#pragma unroll
                for (int c = NC - 1; c > 0; --c) aw[c] = aw[c - 1];
                aw[0] = an[u];
            }
        }
        // T_k for k = k0 + NC - 1 down to k0
        uint64_t T = 0;
        for (int j = k0 + NC; j < WI; ++j) T += B[j];
        uint64_t Tk[NC];
        for (int c = NC - 1; c >= 0; --c) {
            Tk[c] = T;
            T += B[k0 + c];
        }
        int64_t carry = 0;
        for (int c = 0; c < NC; ++c) {
            const uint64_t hi = (acc[c] >> 32) + ((uint64_t)cy[c] << 32);
            const int64_t v = carry + (int64_t)(uint32_t)acc[c] + (int64_t)(uint32_t)Tk[c];
            out[c] = (uint32_t)v;
            carry = (v >> 32) + (int64_t)hi + (int64_t)(Tk[c] >> 32) - (int64_t)Tk[c];
        }
        return carry;
    }

    // adds the column carries of the G column groups into the product's limbs
    // (carry w enters limb (w+1) NC; the last one lands on 2^N') and
    // normalises
    TFT_NEST_HD static void settle_columns(uint32_t *c, const int64_t (&cw)[G]) {
        int64_t carry = 0;
        for (int m0 = NC; m0 < WI; m0 += 4) {
            uint32_t v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = c[m0 + u];
            if (m0 % NC == 0) carry += cw[m0 / NC - 1];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t acc = (int64_t)v[u] + carry;
                v[u] = (uint32_t)acc;
                carry = acc >> 32;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) c[m0 + u] = v[u];
        }
        normalize(c, carry + cw[G - 1]);
    }
};

}  // namespace nest
}  // namespace tft
