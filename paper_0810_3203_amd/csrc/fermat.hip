// HIP kernels for R = Z/(2^N+1) on gfx950: the leaf executor of the
// cache-friendly TFT/ITFT (Alg. 1, Alg. 2), the pointwise products of Sect. 2,
// and the packing of Z[x] coefficients into R (Sect. 5.1).
#include <hip/hip_runtime.h>

#include "desc.hpp"
#include "fermat_dev.hpp"
#include "fermat_leaf.hpp"
#include "fermat_nested.hpp"
#include "kernels.hpp"

namespace tft {

namespace {


// ---------------------------------------------------------------------------
// pointwise products  c = a b 2^scale_e  in Z/(2^N+1)
//
// One workgroup per product.  The negacyclic limb convolution
//   d_k = sum_{j<=k} b_j a_{k-j} - sum_{j>k} b_j a_{k-j+W}          (2^N = -1)
// is computed without a sign test per product: with the doubled array
// A2 = [a_0..a_{W-1}, ~a_0..~a_{W-1}] (~a = 2^32 - 1 - a) and the suffix sums
// T_k = sum_{j>k} b_j,
//   d_k = S_k + T_k - 2^32 T_k,   S_k = sum_{j<W} b_j A2[(k - j) mod 2W],
// where S_k is a sum of unsigned products accumulated in 96 bits.  Each thread
// owns NC consecutive columns and slides a register window over A2.  The
// positive parts S_k + T_k and negative parts 2^32 T_k are then folded into
// four limb vectors that one wave adds with the chunk chains, followed by
// canonicalisation and the multiplication by 2^scale_e.
// ---------------------------------------------------------------------------

// Four columns of the MAC loop: acc[c] += aw[c] bj (64-bit, the carry out of
// each multiply-add into its own SGPR pair), then cy[c] += that carry.  Two
// instructions per limb product; written as instructions because the compiler
// otherwise rebuilds the 64-bit sum with compares and selects.  The four
// multiply-adds come first, so three instructions separate each carry write
// from its read (the VALU SGPR-write to carry-read hazard needs two).
// Registers only (no memory access).
template <int C0, int NC>
__device__ __forceinline__ void mac4(uint64_t (&acc)[NC], uint32_t (&cy)[NC], const uint32_t (&aw)[NC], uint32_t bj) {
    uint64_t c0, c1, c2, c3;
    asm("v_mad_u64_u32 %0, %4, %8, %12, %0\n\t"
        "v_mad_u64_u32 %1, %5, %9, %12, %1\n\t"
        "v_mad_u64_u32 %2, %6, %10, %12, %2\n\t"
        "v_mad_u64_u32 %3, %7, %11, %12, %3"
        : "+v"(acc[C0]), "+v"(acc[C0 + 1]), "+v"(acc[C0 + 2]), "+v"(acc[C0 + 3]), "=&s"(c0), "=&s"(c1), "=&s"(c2),
          "=&s"(c3)
        : "v"(aw[C0]), "v"(aw[C0 + 1]), "v"(aw[C0 + 2]), "v"(aw[C0 + 3]), "v"(bj));
    asm("v_addc_co_u32_e64 %0, %4, %0, 0, %4\n\t"
        "v_addc_co_u32_e64 %1, %5, %1, 0, %5\n\t"
        "v_addc_co_u32_e64 %2, %6, %2, 0, %6\n\t"
        "v_addc_co_u32_e64 %3, %7, %3, 0, %7"
        : "+v"(cy[C0]), "+v"(cy[C0 + 1]), "+v"(cy[C0 + 2]), "+v"(cy[C0 + 3]), "+s"(c0), "+s"(c1), "+s"(c2), "+s"(c3));
}

// threads of a pointwise workgroup for W limbs (64..256) and columns per thread
constexpr uint32_t pw_threads(int W) {
    uint32_t t = (uint32_t)W / 8u;
    t = t < 64 ? 64 : (t > 256 ? 256 : t);
    return (t + 63) / 64 * 64;
}
constexpr int pw_cols(int W) { return W / (int)pw_threads(W) > 0 ? W / (int)pw_threads(W) : 1; }
// LDS words of a pointwise workgroup: A2 (2W), B (W), six column-word arrays (6W)
constexpr uint32_t pw_lds_words(int W) { return 9u * (uint32_t)W; }

// Last phase of a product: with the four limb arrays of LDS filled (A[j] and
// Bv[j] the low words of the positive and negative sums landing on limb j,
// P0[j] and N0[j] their high words, landing on limb j + 1), one wave adds
// them with the chunk chains, takes the residue mod 2^N+1 and multiplies by
// 2^scale_e; special = a or b is 2^N, with A and Bv then holding a and b.
// The result is staged at the start of LDS (W + 1 words) before its store.
// Called by a whole workgroup.
template <int S, int C, bool TR>
__device__ __forceinline__ void pointwise_finish(bool special, uint32_t ta, uint32_t tb, const uint32_t *A,
                                                 const uint32_t *Bv, const uint32_t *P0, const uint32_t *N0,
                                                 uint32_t *c, uint32_t *tc, uint32_t scale_e) {
    using F = FChunk<S, C>;
    constexpr int W = F::W;
    extern __shared__ uint32_t sm[];
    uint32_t *Y = sm;
    uint32_t &topY = Y[F::ESZ];
    const uint32_t tid = threadIdx.x, nthr = blockDim.x;
    if (tid < 64) {
        const FermatOps<F> Bo;
        if (Bo.lane < (uint32_t)S) {  // segment 0 only
            uint32_t s3[C];
            uint32_t top;
            if (!special) {
                uint32_t pl[C], hp[C], nl[C], hn[C], s1[C], s2[C];
#pragma unroll
                for (int j = 0; j < C; ++j) {
                    const uint32_t k = Bo.l * C + j;
                    pl[j] = A[k];
                    nl[j] = Bv[k];
                    hp[j] = k ? P0[k - 1] : N0[W - 1];
                    hn[j] = k ? N0[k - 1] : P0[W - 1];
                }
                const uint32_t c1 = Bo.add(s1, pl, hp);
                const uint32_t b2 = Bo.sub(s2, s1, nl);
                const uint32_t b3 = Bo.sub(s3, s2, hn);
                top = Bo.canon(s3, (int)c1 - (int)b2 - (int)b3, 0, 0u);
            } else if (ta && tb) {
                // (-1)(-1) = 1
#pragma unroll
                for (int j = 0; j < C; ++j) s3[j] = 0u;
                top = Bo.canon(s3, -1, 0, 0u);
            } else {
                // (-1) v = 2^N + 1 - v = ~v + 2
                const uint32_t *v = ta ? Bv : A;
#pragma unroll
                for (int j = 0; j < C; ++j) s3[j] = ~v[Bo.l * C + j];
                top = Bo.canon(s3, -2, 0, 0u);
            }
            Bo.st(Y, s3);
            if (scale_e)
                Bo.twist_store(Y, &topY, scale_e, (int)top);
            else if (Bo.l == 0u)
                topY = top;
        }
    }
    __syncthreads();
    for (uint32_t q = tid; q < (uint32_t)W; q += nthr) c[q] = Y[TR ? q : F::addr(q)];
    if (tid == 0) *tc = topY;
}

// c = a b 2^scale_e for one product; a, b, c are W-limb cells (c may alias a or b),
// ta, tb their top words, tc where c's top goes.  Called by a whole workgroup.
template <int S, int C, bool TR>
__device__ __forceinline__ void pointwise_body(const uint32_t *a, uint32_t ta, const uint32_t *b, uint32_t tb,
                                               uint32_t *c, uint32_t *tc, uint32_t scale_e) {
    using F = FChunk<S, C>;
    constexpr int W = F::W;
    constexpr int NC = pw_cols(W);
    extern __shared__ uint32_t sm[];
    uint32_t *A = sm, *Bv = A + 2 * W;
    uint32_t *P0 = Bv + W, *P1 = P0 + W, *P2 = P1 + W, *N0 = P2 + W, *N1 = N0 + W, *N2 = N1 + W;
    const uint32_t tid = threadIdx.x, nthr = blockDim.x;

    for (uint32_t q = tid; q < (uint32_t)W; q += nthr) {
        const uint32_t g = TR ? F::addr(q) : q;  // global position of limb q
        const uint32_t av = a[g];
        A[q] = av;
        A[q + W] = ~av;
        Bv[q] = b[g];
    }
    __syncthreads();

    const bool special = (ta | tb) != 0u;
    if (!special) {
        // suffix sums T_k = sum_{j>k} b_j (64-bit) in P0 (low) / P1 (high): a doubling scan over W words
        for (uint32_t q = tid; q < (uint32_t)W; q += nthr) {
            P0[q] = q + 1 < (uint32_t)W ? Bv[q + 1] : 0u;
            P1[q] = 0u;
        }
        __syncthreads();
        constexpr int NQ = (W + (int)pw_threads(W) - 1) / (int)pw_threads(W);  // words per thread
        for (uint32_t d = 1; d < (uint32_t)W; d <<= 1) {
            uint64_t add[NQ];
            uint32_t na = 0;
            for (uint32_t q = tid; q < (uint32_t)W; q += nthr, ++na)
                add[na] = q + d < (uint32_t)W ? ((uint64_t)P1[q + d] << 32 | P0[q + d]) : 0ull;
            __syncthreads();
            na = 0;
            for (uint32_t q = tid; q < (uint32_t)W; q += nthr, ++na) {
                const uint64_t t = ((uint64_t)P1[q] << 32 | P0[q]) + add[na];
                P0[q] = (uint32_t)t;
                P1[q] = (uint32_t)(t >> 32);
            }
            __syncthreads();
        }
        // column sums S_k = 2^32 hi + lo: NC consecutive columns per thread.  Each
        // step t = a b + lo fits in 64 bits ((2^32-1)^2 + 2^32-1 < 2^64): lo keeps
        // its low word, hi (64 bits) gathers the high words; no carry tests.
        uint64_t hi[NC], Tk[NC];
        uint32_t lo[NC];
        const uint32_t k0 = tid * NC;
        const bool mine = k0 < (uint32_t)W;
        if (mine) {
            uint32_t aw[NC];
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) {
                lo[cc] = 0;
                hi[cc] = 0;
                aw[cc] = A[k0 + cc];  // window at j = 0: A2[k0 + cc]
                Tk[cc] = (uint64_t)P1[k0 + cc] << 32 | P0[k0 + cc];
            }
            if constexpr (NC % 4 == 0) {
                // S_k = acc + 2^64 cy: 64-bit sums of the products and a count of their wraps
                uint64_t acc[NC];
                uint32_t cy[NC];
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) {
                    acc[cc] = 0;
                    cy[cc] = 0;
                }
#pragma unroll NC
                for (uint32_t j = 0; j < (uint32_t)W; ++j) {
                    const uint32_t bj = Bv[j];
                    static_for<0, NC / 4>([&](auto qc) { mac4<4 * decltype(qc)::value, NC>(acc, cy, aw, bj); });
#pragma unroll
                    for (int cc = NC - 1; cc > 0; --cc) aw[cc] = aw[cc - 1];
                    aw[0] = A[(k0 - j - 1u) & (2u * W - 1u)];
                }
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) {
                    lo[cc] = (uint32_t)acc[cc];
                    hi[cc] = (acc[cc] >> 32) + ((uint64_t)cy[cc] << 32);
                }
            } else {
                // unrolled by the window width so that the slide below is register renaming
#pragma unroll NC
                for (uint32_t j = 0; j < (uint32_t)W; ++j) {
                    const uint64_t bj = Bv[j];
#pragma unroll
                    for (int cc = 0; cc < NC; ++cc) {
                        const uint64_t t = aw[cc] * bj + lo[cc];
                        lo[cc] = (uint32_t)t;
                        hi[cc] += t >> 32;
                    }
                    // slide: the next j needs A2[(k0 + cc - j - 1) mod 2W]
#pragma unroll
                    for (int cc = NC - 1; cc > 0; --cc) aw[cc] = aw[cc - 1];
                    aw[0] = A[(k0 - j - 1u) & (2u * W - 1u)];
                }
            }
        }
        __syncthreads();  // every thread has read its T_k out of P0/P1
        if (mine) {
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) {
                const uint32_t k = k0 + cc;
                // positive part S_k + T_k (96 bits), negative part 2^32 T_k
                const uint64_t w0 = (uint64_t)lo[cc] + (uint32_t)Tk[cc];
                const uint64_t w1 = (hi[cc] & 0xFFFFFFFFull) + (Tk[cc] >> 32) + (w0 >> 32);
                P0[k] = (uint32_t)w0;
                P1[k] = (uint32_t)w1;
                P2[k] = (uint32_t)(hi[cc] >> 32) + (uint32_t)(w1 >> 32);
                N0[k] = 0u;
                N1[k] = (uint32_t)Tk[cc];
                N2[k] = (uint32_t)(Tk[cc] >> 32);
            }
        }
        __syncthreads();
        // fold words of weight 2^(32(k+w)) onto limb positions (2^N = -1)
        constexpr uint32_t T = pw_threads(W);
        constexpr int NS = (W + (int)T - 1) / (int)T;
        uint64_t posv[NS], negv[NS];
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) {
            const uint32_t j = tid + (uint32_t)sl * T;
            uint64_t pos = 0, neg = 0;
            if (j < (uint32_t)W) {
#pragma unroll
                for (uint32_t w = 0; w < 3; ++w) {
                    const uint32_t k = (j + 3u * W - w) % (uint32_t)W;
                    const uint32_t wraps = (k + w) / (uint32_t)W;
                    const uint32_t pw = w == 0 ? P0[k] : (w == 1 ? P1[k] : P2[k]);
                    const uint32_t nw = w == 0 ? N0[k] : (w == 1 ? N1[k] : N2[k]);
                    if (wraps & 1u) {
                        pos += nw;
                        neg += pw;
                    } else {
                        pos += pw;
                        neg += nw;
                    }
                }
            }
            posv[sl] = pos;
            negv[sl] = neg;
        }
        __syncthreads();
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) {
            const uint32_t j = tid + (uint32_t)sl * T;
            if (j < (uint32_t)W) {
                A[j] = (uint32_t)posv[sl];           // PL
                Bv[j] = (uint32_t)negv[sl];          // NL
                P0[j] = (uint32_t)(posv[sl] >> 32);  // PHI (lands at j+1)
                N0[j] = (uint32_t)(negv[sl] >> 32);  // NHI (lands at j+1)
            }
        }
        __syncthreads();
    }

    pointwise_finish<S, C, TR>(special, ta, tb, A, Bv, P0, N0, c, tc, scale_e);
}

// c = a b 2^scale_e for one product through one more Schoenhage-Strassen
// level (fermat_nested.hpp), for W with a nest::Cfg; a and b not 2^N.
// kNestThreads threads: the transforms give every lane a digit of a
// butterfly; the inner products give each wave a group of columns of all K
// products (a lane a product); carries are resolved a lane a cell.
constexpr uint32_t kNestThreads = 256;

// forward transform of the digit cells D (cell pitch WI + 1 int64): item =
// (butterfly, digit); every item reads before any writes
template <class NS>
__device__ __forceinline__ void nested_forward(int64_t *D, uint32_t tid) {
    constexpr int K = NS::K, WI = NS::WI, CP = WI + 1;
    constexpr uint32_t T = kNestThreads, HW = (uint32_t)(K / 2 * WI), FI = (HW + T - 1u) / T;
    for (int hs = K / 2; hs >= 1; hs >>= 1) {
        int64_t sv[FI], ev[FI];
        uint32_t xi[FI], yi[FI];
#pragma unroll
        for (uint32_t k = 0; k < FI; ++k) {
            const uint32_t e = tid + k * T;
            xi[k] = ~0u;
            if (e < HW) {
                const uint32_t t = e / WI, d = e - t * WI;
                const uint32_t off = t % (uint32_t)hs, o = (t / (uint32_t)hs) * 2u * hs + off;
                const int64_t x = D[o * CP + d], y = D[(o + hs) * CP + d];
                uint32_t dd = d + (uint32_t)NS::twiddle_limbs((int)off, hs);
                int64_t dv = x - y;
                if (dd >= (uint32_t)WI) {  // past 2^N' = -1
                    dd -= WI;
                    dv = -dv;
                }
                sv[k] = x + y;
                ev[k] = dv;
                xi[k] = o * CP + d;
                yi[k] = (o + hs) * CP + dd;
            }
        }
        __syncthreads();
#pragma unroll
        for (uint32_t k = 0; k < FI; ++k)
            if (xi[k] != ~0u) {
                D[xi[k]] = sv[k];
                D[yi[k]] = ev[k];
            }
        __syncthreads();
    }
}

template <int S, int C, bool TR>
__device__ __forceinline__ void nested_body(const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t *tc,
                                            uint32_t scale_e) {
    using F = FChunk<S, C>;
    constexpr int W = F::W;
    using NS = nest::Nest<W>;
    constexpr int K = NS::K, WI = NS::WI, WP = NS::WP, NC = NS::NC, G = NS::G, CP = WI + 1, DP = NS::DP;
    constexpr uint32_t T = kNestThreads, KW = (uint32_t)(K * WI), HW = (uint32_t)(K / 2 * WI);
    static_assert(G * 64 == (int)T, "a wave per column group");
    extern __shared__ uint32_t sm[];
    int64_t *D = reinterpret_cast<int64_t *>(sm + NS::D);
    uint32_t *LA = sm + NS::LA, *CWS = sm + NS::CW;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;

    // a: split, transform, normalise into LA.  The split takes lane = cell
    // and wave = a range of piece limbs: in the transposed layout limb k of
    // the K pieces is one contiguous row, so each load is a whole row.
    constexpr int KPW = NS::PL / G, DPW = (WI + G - 1) / G;
    static_assert(KPW * G == NS::PL, "piece limbs split evenly over the waves");
    auto split = [&](const uint32_t *x) {
        auto limb = [&](int q) { return x[TR ? F::addr((uint32_t)q) : (uint32_t)q]; };
        int64_t *cell = D + lane * CP;
        const int d0 = (int)wave * DPW, d1 = d0 + DPW < WI ? d0 + DPW : WI;
        NS::split_zero((int)lane, d0, d1, cell);
        NS::split_part(limb, (int)lane, (int)wave * KPW, ((int)wave + 1) * KPW, cell);
    };
    split(a);
    __syncthreads();
    nested_forward<NS>(D, tid);
    if (wave == 0u) NS::norm_digits(D + lane * CP, LA + lane * WP);
    __syncthreads();
    // b: the same, normalised in place in the digit region
    split(b);
    __syncthreads();
    nested_forward<NS>(D, tid);
    if (wave == 0u) NS::norm_digits(D + lane * CP, sm + NS::D + lane * DP);
    __syncthreads();
    // inner products: lane = position, wave = column group
    uint32_t *Ai = LA + lane * WP;
    const uint32_t *Bi = sm + NS::D + lane * DP;
    const bool sp = NS::geth(Ai) != 0 || NS::geth(Bi) != 0;
    uint32_t out[NC];
    const int64_t cw = NS::columns(Ai, Bi, (int)wave * NC, out,
                                   [](uint64_t (&acc)[NC], uint32_t (&cy)[NC], const uint32_t (&aw)[NC], uint32_t bj) {
                                       static_for<0, NC / 4>(
                                           [&](auto qc) { mac4<4 * decltype(qc)::value, NC>(acc, cy, aw, bj); });
                                   });
    __syncthreads();  // every wave has read its A columns
    if (!sp) {
#pragma unroll
        for (int k = 0; k < NC; ++k) Ai[(int)wave * NC + k] = out[k];
    }
    CWS[2u * (wave * 64u + lane)] = (uint32_t)cw;
    CWS[2u * (wave * 64u + lane) + 1u] = (uint32_t)((uint64_t)cw >> 32);
    __syncthreads();
    if (wave == 0u) {
        if (sp) {
            NS::special_product(Ai, Bi, Ai);
        } else {
            int64_t cws[G];
#pragma unroll
            for (int w = 0; w < G; ++w)
                cws[w] = (int64_t)((uint64_t)CWS[2u * (w * 64u + lane) + 1u] << 32 | CWS[2u * (w * 64u + lane)]);
            NS::settle_columns(Ai, cws);
        }
    }
    __syncthreads();
    // products as digit cells (value L + h 2^N' = L - h)
    for (uint32_t e = tid; e < KW; e += T) {
        const uint32_t i = e / WI, d = e - i * WI;
        int64_t v = LA[i * WP + d];
        if (d == 0u) v -= NS::geth(LA + i * WP);
        D[i * CP + d] = v;
    }
    __syncthreads();
    // inverse transform: item = (butterfly, digit); t = y w^-off has digit d
    // from y's digit d + q (negated past 2^N')
    constexpr uint32_t II = (HW + T - 1u) / T;
    for (int hs = 1; hs <= K / 2; hs <<= 1) {
        int64_t xv[II], yv[II];
        uint32_t xi[II], yi[II];
#pragma unroll
        for (uint32_t k = 0; k < II; ++k) {
            const uint32_t e = tid + k * T;
            xi[k] = ~0u;
            if (e < HW) {
                const uint32_t t = e / WI, d = e - t * WI;
                const uint32_t off = t % (uint32_t)hs, o = (t / (uint32_t)hs) * 2u * hs + off;
                const int64_t x = D[o * CP + d];
                const uint32_t dq = d + (uint32_t)NS::twiddle_limbs((int)off, hs);
                const int64_t y = dq < (uint32_t)WI ? D[(o + hs) * CP + dq] : -D[(o + hs) * CP + dq - WI];
                xv[k] = x + y;
                yv[k] = x - y;
                xi[k] = o * CP + d;
                yi[k] = (o + hs) * CP + d;
            }
        }
        __syncthreads();
#pragma unroll
        for (uint32_t k = 0; k < II; ++k)
            if (xi[k] != ~0u) {
                D[xi[k]] = xv[k];
                D[yi[k]] = yv[k];
            }
        __syncthreads();
    }
    if (wave == 0u) NS::norm_digits(D + lane * CP, Ai);
    __syncthreads();
    // untwist and 1/K into the digit cells, then the signed coefficients
    for (uint32_t e = tid; e < KW; e += T) {
        const uint32_t i = e / WI, d = e - i * WI;
        D[i * CP + d] = NS::untwist_digit(LA + i * WP, (int)i, (int)d);
    }
    __syncthreads();
    if (wave == 0u) {
        NS::norm_digits(D + lane * CP, Ai);
        NS::magnitude(Ai, Ai);
    }
    __syncthreads();
    // per-limb positive / negative sums in the last phase's arrays
    for (uint32_t j = tid; j < (uint32_t)W; j += T) {
        uint64_t pos, neg;
        NS::gather(LA, (int)j, pos, neg);
        sm[NS::PA + j] = (uint32_t)pos;
        sm[NS::PB + j] = (uint32_t)neg;
        sm[NS::P0 + j] = (uint32_t)(pos >> 32);
        sm[NS::N0 + j] = (uint32_t)(neg >> 32);
    }
    __syncthreads();
    pointwise_finish<S, C, TR>(false, 0u, 0u, sm + NS::PA, sm + NS::PB, sm + NS::P0, sm + NS::N0, c, tc, scale_e);
}

// waves a SIMD the register budget is sized for: two workgroups share a
// compute unit up to 2048 limbs; at 4096 limbs the LDS holds one, and the
// registers are not capped
template <int W>
constexpr int nest_min_waves() {
    return W >= 4096 ? 1 : 2;
}

template <int S, int C, bool TR>
__global__ void __launch_bounds__(kNestThreads, nest_min_waves<S * C>()) fermat_pointwise_nested_kernel(const uint32_t *__restrict__ a,
                                                                      const uint32_t *__restrict__ b, uint32_t *c,
                                                                      uint64_t cap, uint32_t scale_e, uint32_t base) {
    constexpr int W = S * C;
    const uint64_t i = (uint64_t)base + blockIdx.x;
    const uint32_t ta = a[cap * W + i], tb = b[cap * W + i];
    if ((ta | tb) != 0u)
        pointwise_body<S, C, TR>(a + i * W, ta, b + i * W, tb, c + i * W, c + cap * W + i, scale_e);
    else
        nested_body<S, C, TR>(a + i * W, b + i * W, c + i * W, c + cap * W + i, scale_e);
}

template <int S, int C, bool TR>
__global__ void __launch_bounds__(kNestThreads, nest_min_waves<S * C>()) fermat_pointwise_nested_items_kernel(uint32_t *x, uint64_t cap,
                                                                            const uint4 *__restrict__ items) {
    constexpr int W = S * C;
    const uint4 it = items[blockIdx.x];
    uint32_t *ca = x + (uint64_t)it.x * W, *cb = x + (uint64_t)it.y * W;
    const uint32_t ta = x[cap * W + it.x], tb = x[cap * W + it.y];
    if ((ta | tb) != 0u)
        pointwise_body<S, C, TR>(ca, ta, cb, tb, ca, x + cap * W + it.x, it.z);
    else
        nested_body<S, C, TR>(ca, cb, ca, x + cap * W + it.x, it.z);
}

template <int S, int C, bool TR>
__global__ void __launch_bounds__(256) fermat_pointwise_kernel(const uint32_t *__restrict__ a,
                                                               const uint32_t *__restrict__ b, uint32_t *c,
                                                               uint64_t cap, uint32_t scale_e, uint32_t base) {
    constexpr int W = S * C;
    const uint64_t i = (uint64_t)base + blockIdx.x;
    pointwise_body<S, C, TR>(a + i * W, a[cap * W + i], b + i * W, b[cap * W + i], c + i * W, c + cap * W + i,
                             scale_e);
}

// Pointwise products over a list: item i multiplies cells it.x and it.y of the
// cell array x (capacity cap) into cell it.x, with its own scale 2^it.z.
template <int S, int C, bool TR>
__global__ void __launch_bounds__(256) fermat_pointwise_items_kernel(uint32_t *x, uint64_t cap,
                                                                     const uint4 *__restrict__ items) {
    constexpr int W = S * C;
    const uint4 it = items[blockIdx.x];
    uint32_t *ca = x + (uint64_t)it.x * W, *cb = x + (uint64_t)it.y * W;
    pointwise_body<S, C, TR>(ca, x[cap * W + it.x], cb, x[cap * W + it.y], ca, x + cap * W + it.x, it.z);
}

// Pack: cell e of an operand holds coefficients e*k .. e*k+k-1, coefficient
// e*k+j in limbs [j*ws, j*ws + climbs) (slot j), zeros elsewhere (Sect. 5.1 with
// k = 1; k > 1 bundles k coefficients per ring element).  One descriptor per
// operand, blockIdx.y selects it.
// Position of limb k of a W-limb cell in the transposed layout (W = 64 C >= 128),
// and its inverse; identity for W <= 64.
__device__ __forceinline__ uint32_t tpos(uint32_t k, uint32_t W) {
    const uint32_t C = W >> 6;
    return C > 1 ? (k & (C - 1)) * 64u + k / C : k;
}
__device__ __forceinline__ uint32_t tlimb(uint32_t p, uint32_t W) {
    const uint32_t C = W >> 6;
    return C > 1 ? (p & 63u) * C + (p >> 6) : p;
}

__global__ void fermat_pack_kernel(const PackDesc *__restrict__ descs, PackDesc inl, uint32_t *__restrict__ x,
                                   uint64_t cap, uint32_t W, uint32_t tr) {
    const PackDesc d = descs ? descs[blockIdx.y] : inl;
    const uint64_t total = d.z * (uint64_t)W;
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < total;
         q += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t e = q / W;
        const uint32_t p = (uint32_t)(q % W);
        const uint32_t k = tr ? tlimb(p, W) : p;  // limb held at position p
        const uint32_t j = k / d.ws, off = k % d.ws;
        const uint64_t c = e * d.k + j;
        x[(d.cell0 + e) * W + p] = (j < d.k && off < d.climbs && c < d.len) ? d.coef[c * d.climbs + off] : 0u;
        if (p == 0) x[cap * W + d.cell0 + e] = 0u;
    }
}

// The same for transposed cells of 1024 limbs and more: one workgroup a cell
// reads the cell's limbs in their natural order (each slot a contiguous run of
// a coefficient) into LDS, then writes the cell in transposed order.  LDS word
// k + k/C holds limb k, so the reads at stride C limbs of the second loop hit
// distinct banks.  The plain kernel reads limb tlimb(p) for position p, C
// limbs from its neighbour's, a different cache line per lane.
__global__ void __launch_bounds__(256) fermat_pack_rows_kernel(const PackDesc *__restrict__ descs, PackDesc inl,
                                                               uint32_t *__restrict__ x, uint64_t cap, uint32_t W) {
    const PackDesc d = descs ? descs[blockIdx.y] : inl;
    extern __shared__ uint32_t sm[];
    const uint32_t C = W >> 6;
    for (uint64_t e = blockIdx.x; e < d.z; e += gridDim.x) {
        __syncthreads();  // the previous cell's reads of sm are done
        for (uint32_t k = threadIdx.x; k < W; k += blockDim.x) {
            const uint32_t j = k / d.ws, off = k % d.ws;
            const uint64_t c = e * d.k + j;
            sm[k + k / C] = (j < d.k && off < d.climbs && c < d.len) ? d.coef[c * d.climbs + off] : 0u;
        }
        __syncthreads();
        uint32_t *dst = x + (d.cell0 + e) * W;
        for (uint32_t p = threadIdx.x; p < W; p += blockDim.x) {
            const uint32_t k = tlimb(p, W);
            dst[p] = sm[k + k / C];
        }
        if (threadIdx.x == 0) x[cap * W + d.cell0 + e] = 0u;
    }
}

// Unpack with k = 1: coefficient t is the low limbs of cell t.
__global__ void fermat_unpack1_kernel(const UnpackDesc *__restrict__ descs, UnpackDesc inl,
                                      const uint32_t *__restrict__ x, uint64_t cap, uint32_t W, uint32_t tr) {
    const UnpackDesc d = descs ? descs[blockIdx.y] : inl;
    const uint64_t total = d.len_out * (uint64_t)d.olimbs;
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < total;
         q += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t t = q / d.olimbs;
        const uint32_t i = (uint32_t)(q % d.olimbs);
        const uint64_t cell = d.cell0 + t;
        d.out[q] = i < W ? x[cell * W + (tr ? tpos(i, W) : i)] : (i == W ? x[cap * W + cell] : 0u);
    }
}

// The same for transposed cells whose output row takes most of the cell: one
// workgroup a coefficient reads its cell contiguously into LDS (rows of 64
// words padded to 65, so the column reads below hit distinct banks), then
// writes the output row contiguously.  The plain kernel reads limb i at
// transposed position tpos(i), 256 bytes from limb i+1, so each of its loads
// touches a different cache line per lane.
__global__ void __launch_bounds__(256) fermat_unpack1_rows_kernel(const UnpackDesc *__restrict__ descs,
                                                                  UnpackDesc inl, const uint32_t *__restrict__ x,
                                                                  uint64_t cap, uint32_t W) {
    const UnpackDesc d = descs ? descs[blockIdx.y] : inl;
    extern __shared__ uint32_t sm[];
    const uint32_t C = W >> 6;
    for (uint64_t t = blockIdx.x; t < d.len_out; t += gridDim.x) {
        const uint64_t cell = d.cell0 + t;
        const uint32_t *src = x + cell * W;
        __syncthreads();  // the previous coefficient's reads of sm are done
        for (uint32_t p = threadIdx.x; p < W; p += blockDim.x) sm[(p >> 6) * 65u + (p & 63u)] = src[p];
        __syncthreads();
        uint32_t *o = d.out + t * d.olimbs;
        for (uint32_t i = threadIdx.x; i < d.olimbs; i += blockDim.x)
            o[i] = i < W ? sm[(i & (C - 1u)) * 65u + i / C] : (i == W ? x[cap * W + cell] : 0u);
    }
}

// Unpack with k > 1: the product cell m holds slots 0..2k-2 of width ws limbs;
// coefficient t = m k + j is slot j of cell m plus slot j + k of cell m - 1.
// One wave per coefficient and a lane per limb (64 limbs per round): limb i is
// v_i = s0_i + s1_i (< 2^33 - 1, so it emits at most one carry) plus the carry
// from the limbs below.  With G the lanes whose v_i carries out, P the lanes
// whose low word is all ones (they pass a carry on) and c the carry into the
// round, the carries into the lanes are the bits of (a + G + c) ^ a ^ G with
// a = G | P, and the carry out of the round is that sum's overflow.  Loads of
// one slot and the output row are contiguous per wave.
__global__ void __launch_bounds__(256) fermat_unpackk_kernel(const UnpackDesc *__restrict__ descs, UnpackDesc inl,
                                                             const uint32_t *__restrict__ x, uint32_t W,
                                                             uint32_t tr) {
    const UnpackDesc d = descs ? descs[blockIdx.y] : inl;
    const uint32_t lane = threadIdx.x & 63u, wpb = blockDim.x >> 6;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint64_t t = (uint64_t)blockIdx.x * wpb + wave; t < d.len_out; t += (uint64_t)gridDim.x * wpb) {
        const uint64_t m = t / d.k;
        const uint32_t j = (uint32_t)(t % d.k);
        // slot j of cell m and slot j + k of cell m - 1 (limbs j ws + i, (j + k) ws + i)
        const bool h0 = m < d.ncells, h1 = m >= 1 && j + 1 < d.k && m - 1 < d.ncells;
        const uint32_t *s0 = x + (d.cell0 + m) * W;
        const uint32_t *s1 = h1 ? x + (d.cell0 + m - 1) * W : x;
        const uint32_t k0 = j * d.ws, k1 = (j + d.k) * d.ws;
        uint32_t *o = d.out + t * d.olimbs;
        uint64_t c = 0;
        for (uint32_t i0 = 0; i0 < d.olimbs; i0 += 64u) {
            const uint32_t i = i0 + lane;
            uint64_t v = 0;
            if (i < d.ws) {
                if (h0) v += s0[tr ? tpos(k0 + i, W) : k0 + i];
                if (h1) v += s1[tr ? tpos(k1 + i, W) : k1 + i];
            }
            const uint32_t lo = (uint32_t)v;
            const uint64_t G = ballot((v >> 32) != 0ull), P = ballot(lo == 0xFFFFFFFFu);
            const uint64_t a = G | P, s = a + G, s2 = s + c;
            const uint64_t cin = s2 ^ a ^ G;
            if (i < d.olimbs) o[i] = lo + (uint32_t)((cin >> lane) & 1ull);
            c = (s < a || s2 < s) ? 1ull : 0ull;
        }
    }
}

template <class KernelT>
hipError_t pointwise_attr(KernelT *kern, size_t lds, bool &done) {
    if (done || lds <= 65536) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
    if (e == hipSuccess) done = true;
    return e;
}

// W with a nest::Cfg take the nested product (one more SS level); measured
// faster than the schoolbook kernel at every one of them (16384 to 131072
// bits: 1.2x, 1.3x, 2.6x, 3.8x on 20000 products)
template <int W>
constexpr bool pw_nested() {
    return W == 512 || W == 1024 || W == 2048 || W == 4096;
}

template <int W>
constexpr size_t pw_lds_bytes() {
    if constexpr (pw_nested<W>()) {
        constexpr size_t n = (size_t)nest::Nest<W>::WORDS, s = (size_t)pw_lds_words(W);
        return 4 * (n > s ? n : s);  // the special operands take the schoolbook path's layout
    } else {
        return (size_t)pw_lds_words(W) * 4;
    }
}

template <int W>
constexpr uint32_t pw_block() {
    return pw_nested<W>() ? kNestThreads : pw_threads(W);
}

template <int S, int C, bool TR>
auto pw_kernel() {
    if constexpr (pw_nested<S * C>())
        return &fermat_pointwise_nested_kernel<S, C, TR>;
    else
        return &fermat_pointwise_kernel<S, C, TR>;
}

template <int S, int C, bool TR>
auto pw_items_kernel() {
    if constexpr (pw_nested<S * C>())
        return &fermat_pointwise_nested_items_kernel<S, C, TR>;
    else
        return &fermat_pointwise_items_kernel<S, C, TR>;
}

template <int S, int C, bool TR>
hipError_t pointwise_launch(uint64_t n, const uint32_t *a, const uint32_t *b, uint32_t *c, uint64_t cap,
                            uint32_t scale_e, hipStream_t st) {
    constexpr int W = S * C;
    constexpr size_t lds = pw_lds_bytes<W>();
    if (lds > kLdsBudget) return hipErrorInvalidValue;
    static bool attr = false;
    auto kern = pw_kernel<S, C, TR>();
    hipError_t e = pointwise_attr(kern, lds, attr);
    if (e != hipSuccess) return e;
    const uint64_t per = kMaxGridX / pw_block<W>();
    for (uint64_t i0 = 0; i0 < n; i0 += per) {
        const uint64_t nb = n - i0 < per ? n - i0 : per;
        hipLaunchKernelGGL(kern, dim3((uint32_t)nb), dim3(pw_block<W>()), lds, st, a, b, c, cap, scale_e, (uint32_t)i0);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int S, int C, bool TR>
hipError_t pointwise_items_launch(uint64_t nitems, uint32_t *x, uint64_t cap, const uint4 *items, hipStream_t st) {
    constexpr int W = S * C;
    constexpr size_t lds = pw_lds_bytes<W>();
    if (lds > kLdsBudget) return hipErrorInvalidValue;
    static bool attr = false;
    auto kern = pw_items_kernel<S, C, TR>();
    hipError_t e = pointwise_attr(kern, lds, attr);
    if (e != hipSuccess) return e;
    const uint64_t per = kMaxGridX / pw_block<W>();
    for (uint64_t i0 = 0; i0 < nitems; i0 += per) {
        const uint64_t nb = nitems - i0 < per ? nitems - i0 : per;
        hipLaunchKernelGGL(kern, dim3((uint32_t)nb), dim3(pw_block<W>()), lds, st, x, cap, items + i0);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

uint32_t lds_budget_bytes() { return kLdsBudget - kLeafStaticLds; }

hipError_t launch_fermat_leaf(uint32_t W, uint32_t nwaves, uint32_t njobs, uint32_t lds_cells, const Job *jobs,
                              uint32_t job_offset, const LeafProg *progs, const LeafStep *steps, const LeafOp *ops,
                              uint32_t *x, uint64_t cap, uint32_t ord_mask, uint32_t opmask, bool transposed,
                              hipStream_t st) {
    if (fermat_leaf2_supported(W))
        return launch_fermat_leaf2(W, njobs, lds_cells, jobs, job_offset, progs, steps, ops, x, cap, ord_mask, opmask,
                                   transposed, st);
    return transposed ? launch_fermat_leaf_trans(W, nwaves, njobs, lds_cells, jobs, job_offset, progs, steps, ops, x,
                                                 cap, ord_mask, opmask, st)
                      : launch_fermat_leaf_plain(W, nwaves, njobs, lds_cells, jobs, job_offset, progs, steps, ops, x,
                                                 cap, ord_mask, opmask, st);
}

uint32_t fermat_lds_cell_bytes(uint32_t W) { return 4u * (W + 1u); }

template <bool TR>
struct PwLaunch {
    template <int S, int C>
    static hipError_t run(uint64_t n, const uint32_t *a, const uint32_t *b, uint32_t *c, uint64_t cap,
                          uint32_t scale_e, hipStream_t st) {
        return pointwise_launch<S, C, TR>(n, a, b, c, cap, scale_e, st);
    }
    template <int S, int C>
    static hipError_t items(uint64_t nitems, uint32_t *x, uint64_t cap, const uint4 *it, hipStream_t st) {
        return pointwise_items_launch<S, C, TR>(nitems, x, cap, it, st);
    }
};

hipError_t launch_fermat_pointwise(uint32_t W, uint64_t n, const uint32_t *a, const uint32_t *b, uint32_t *c,
                                   uint64_t cap, uint32_t scale_e, bool transposed, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (transposed) {
        TFT_FERMAT_DISPATCH(W, PwLaunch<true>::run, n, a, b, c, cap, scale_e, st)
    }
    TFT_FERMAT_DISPATCH(W, PwLaunch<false>::run, n, a, b, c, cap, scale_e, st)
}

hipError_t launch_fermat_pointwise_items(uint32_t W, uint64_t nitems, uint32_t *x, uint64_t cap, const uint4 *items,
                                         bool transposed, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    if (!transposed) return hipErrorInvalidValue;  // products keep their cell arrays transposed
    TFT_FERMAT_DISPATCH(W, PwLaunch<true>::items, nitems, x, cap, items, st)
}

hipError_t launch_fermat_pack(uint32_t W, const PackDesc *descs, uint32_t ndesc, const PackDesc &inl, uint64_t max_z,
                              uint32_t *x, uint64_t cap, bool transposed, hipStream_t st) {
    if (ndesc == 0 || max_z == 0) return hipSuccess;
    // about 8 words per thread for the largest operand: with one grid row per
    // descriptor, rows of small operands would otherwise launch mostly idle blocks
    // cells of 1024 limbs and more through LDS (at 256 limbs the plain kernel
    // is faster: the 4096-request batch took 770 ms against 750 ms)
    if (transposed && W >= 1024u) {
        const uint64_t blocks = max_z < 16384 ? max_z : 16384;
        hipLaunchKernelGGL(fermat_pack_rows_kernel, dim3((uint32_t)blocks, ndesc), dim3(256),
                           (size_t)(W + W / (W / 64u)) * 4u, st, descs, inl, x, cap, W);
        return hipGetLastError();
    }
    uint64_t blocks = (max_z * W + 2047) / 2048;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fermat_pack_kernel, dim3((uint32_t)blocks, ndesc), dim3(256), 0, st, descs, inl, x, cap, W,
                       transposed ? 1u : 0u);
    return hipGetLastError();
}

hipError_t launch_fermat_unpack(uint32_t W, const UnpackDesc *descs, uint32_t ndesc, const UnpackDesc &inl,
                                uint64_t max_len, uint32_t max_olimbs, bool bundled, const uint32_t *x, uint64_t cap,
                                bool transposed, hipStream_t st) {
    if (ndesc == 0 || max_len == 0) return hipSuccess;
    const uint32_t tr = transposed ? 1u : 0u;
    // about 8 words (coefficients) per thread (wave) for the largest product, as in the pack
    if (!bundled && tr && W >= 1024u && 2ull * max_olimbs >= W) {
        // whole cells of 1024 limbs and more through LDS: each output row takes
        // most of its cell
        const uint64_t blocks = max_len < 16384 ? max_len : 16384;
        hipLaunchKernelGGL(fermat_unpack1_rows_kernel, dim3((uint32_t)blocks, ndesc), dim3(256),
                           (size_t)(W / 64u) * 65u * 4u, st, descs, inl, x, cap, W);
    } else if (!bundled) {
        uint64_t blocks = (max_len * max_olimbs + 2047) / 2048;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(fermat_unpack1_kernel, dim3((uint32_t)blocks, ndesc), dim3(256), 0, st, descs, inl, x, cap,
                           W, tr);
    } else {
        uint64_t blocks = (max_len + 31) / 32;  // four waves per block, a wave per coefficient
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(fermat_unpackk_kernel, dim3((uint32_t)blocks, ndesc), dim3(256), 0, st, descs, inl, x, W,
                           tr);
    }
    return hipGetLastError();
}

}  // namespace tft
