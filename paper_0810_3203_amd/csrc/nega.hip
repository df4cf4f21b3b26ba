// HIP kernels for R = (Z/mZ)[y]/(y^K+1), theta = y of order 2K (Sect. 5.2):
// leaf executor of the cache-friendly TFT/ITFT, negacyclic pointwise products,
// and the cutting of (Z/mZ)[x] operands into pieces of K/2 coefficients.
//
// An element is K coefficients in [0, m), m odd < 2^62.  Multiplication by
// y^e is an index rotation with a sign flip of the coefficients that pass
// y^K = -1; the ring needs no carries, so a coefficient is independent work.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "desc.hpp"
#include "nega.hpp"

namespace tft {

namespace {

constexpr uint32_t kLdsBudget = 160u * 1024u;
// work-items per grid dimension of one launch (the dispatch packet holds 32-bit sizes)
constexpr uint32_t kMaxGridX = 0xFFFFFFFFu;

__device__ __forceinline__ uint64_t madd(uint64_t a, uint64_t b, uint64_t m) {
    const uint64_t s = a + b;
    return s >= m ? s - m : s;
}
__device__ __forceinline__ uint64_t msub(uint64_t a, uint64_t b, uint64_t m) { return a >= b ? a - b : a + m - b; }
__device__ __forceinline__ uint64_t mneg(uint64_t a, uint64_t m) { return a ? m - a : 0; }
__device__ __forceinline__ uint64_t mhalf(uint64_t a, uint64_t m) { return (a & 1) ? (a + m) >> 1 : a >> 1; }

template <int S_, int R_>
struct NegaSeg {
    static constexpr int S = S_;
    static constexpr int R = R_;
    static constexpr int K = S * R;
    uint32_t l;
    uint64_t m;

    // coefficient k of y^e * x  (0 <= e < 2K)
    __device__ __forceinline__ uint64_t rot(const uint64_t *x, uint32_t k, uint32_t e) const {
        const uint32_t t = (k - e) & (2u * K - 1u);
        const uint64_t v = x[t & (K - 1u)];
        return (t & (uint32_t)K) ? mneg(v, m) : v;
    }
    __device__ __forceinline__ uint64_t rot_diff(const uint64_t *x0, const uint64_t *x1, uint32_t k,
                                                 uint32_t e) const {
        const uint32_t t = (k - e) & (2u * K - 1u);
        const uint32_t src = t & (K - 1u);
        return (t & (uint32_t)K) ? msub(x1[src], x0[src], m) : msub(x0[src], x1[src], m);
    }

    __device__ void t22(uint64_t *x0, uint64_t *x1, uint32_t e) const {
        uint64_t D[R];
#pragma unroll
        for (int r = 0; r < R; ++r) D[r] = rot_diff(x0, x1, (uint32_t)r * S + l, e);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = (uint32_t)r * S + l;
            x0[k] = madd(x0[k], x1[k], m);
            x1[k] = D[r];
        }
    }
    __device__ void t21(uint64_t *x0, uint64_t *x1, uint32_t e) const {
        uint64_t D[R];
#pragma unroll
        for (int r = 0; r < R; ++r) D[r] = rot(x0, (uint32_t)r * S + l, e);
#pragma unroll
        for (int r = 0; r < R; ++r) x1[(uint32_t)r * S + l] = D[r];
    }
    __device__ void add2(uint64_t *x0, const uint64_t *x1) const {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = (uint32_t)r * S + l;
            x0[k] = madd(x0[k], x1[k], m);
        }
    }
    __device__ void i2(uint64_t *x0, uint64_t *x1, uint32_t einv) const {
        uint64_t V[R];
#pragma unroll
        for (int r = 0; r < R; ++r) V[r] = rot(x1, (uint32_t)r * S + l, einv);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = (uint32_t)r * S + l;
            const uint64_t a = x0[k];
            x0[k] = madd(a, V[r], m);
            x1[k] = msub(a, V[r], m);
        }
    }
    // (x0, x1) <- (2 x0 - x1, y^e (x0 - x1)); z2 = false: x1 taken as 0
    __device__ void i1f1(uint64_t *x0, uint64_t *x1, uint32_t e, bool z2) const {
        uint64_t D[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = (uint32_t)r * S + l;
            D[r] = z2 ? rot_diff(x0, x1, k, e) : rot(x0, k, e);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = (uint32_t)r * S + l;
            const uint64_t a = x0[k];
            x0[k] = z2 ? msub(madd(a, a, m), x1[k], m) : madd(a, a, m);
            x1[k] = D[r];
        }
    }
    __device__ void dbl_sub(uint64_t *x0, const uint64_t *x1) const {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = (uint32_t)r * S + l;
            const uint64_t a = x0[k];
            x0[k] = x1 ? msub(madd(a, a, m), x1[k], m) : madd(a, a, m);
        }
    }
    __device__ void half(uint64_t *x0, const uint64_t *x1) const {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = (uint32_t)r * S + l;
            x0[k] = mhalf(x1 ? madd(x0[k], x1[k], m) : x0[k], m);
        }
    }
};

template <int S, int R>
__global__ void __launch_bounds__(512) nega_leaf_kernel(const Job *__restrict__ jobs,
                                                         const LeafProg *__restrict__ progs,
                                                         const LeafStep *__restrict__ steps,
                                                         const LeafOp *__restrict__ ops, uint64_t *__restrict__ x,
                                                         uint64_t m, uint32_t ord_mask, uint32_t job_offset) {
    constexpr int K = S * R;
    constexpr uint32_t G = 64 / S;
    extern __shared__ uint64_t smq[];
    const Job J = jobs[job_offset + blockIdx.x];
    const LeafProg P = progs[J.prog];
    const uint32_t tid = threadIdx.x, nthr = blockDim.x;
    constexpr uint32_t KQ = K / 2;  // uint4 chunks per cell
    // CB reads of a thread in flight together (a loop that stored each read
    // into LDS before the next would wait for every read in turn).  Past the
    // end a thread reads and stores the last chunk again (the same value at
    // the same place), so neither loop has a branch the reads could sink into.
    constexpr int CB = 8;
    const uint32_t total = J.nload * KQ;
    for (uint32_t q0 = tid; q0 < total; q0 += nthr * CB) {
        uint4 v[CB];
        uint32_t qs[CB];
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            const uint32_t q = q0 + (uint32_t)b * nthr;
            qs[b] = q < total ? q : total - 1u;
            const uint32_t cell = qs[b] / KQ, off = qs[b] % KQ;
            v[b] = reinterpret_cast<const uint4 *>(x + (J.base + (uint64_t)cell * J.stride) * K)[off];
        }
#pragma unroll
        for (int b = 0; b < CB; ++b) reinterpret_cast<uint4 *>(smq)[qs[b]] = v[b];
    }
    __syncthreads();
    NegaSeg<S, R> B;
    const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    B.l = lane & (S - 1);
    B.m = m;
    const uint32_t g = lane / S;
    const uint32_t wave = tid >> 6, nwaves = nthr >> 6;
    for (uint32_t st = 0; st < P.step_count; ++st) {
        const LeafStep LS = steps[P.step_begin + st];
        for (uint32_t jb = wave * G; jb < LS.op_count; jb += nwaves * G) {
            const uint32_t j = jb + g;
            if (j < LS.op_count) {
                const LeafOp o = ops[LS.op_begin + j];
                const uint32_t code = o.w0 & 15u;
                const uint32_t i0 = (o.w0 >> 4) & 16383u, i1 = (o.w0 >> 18) & 16383u;
                const uint32_t e =
                    (uint32_t)((((uint64_t)J.s << op_alog(o)) + (uint64_t)op_b(o)) & ord_mask);
                uint64_t *x0 = smq + (size_t)i0 * K, *x1 = smq + (size_t)i1 * K;
                switch (code) {
                    case OP_T22: B.t22(x0, x1, e); break;
                    case OP_T21: B.t21(x0, x1, e); break;
                    case OP_T12: B.add2(x0, x1); break;
                    case OP_I2: B.i2(x0, x1, (0u - e) & ord_mask); break;
                    case OP_I1F1Z2: B.i1f1(x0, x1, e, true); break;
                    case OP_I1F1Z1: B.i1f1(x0, x1, e, false); break;
                    case OP_I1F0Z2: B.dbl_sub(x0, x1); break;
                    case OP_I1F0Z1: B.dbl_sub(x0, nullptr); break;
                    case OP_I0Z2: B.half(x0, x1); break;
                    case OP_I0Z1: B.half(x0, nullptr); break;
                    default: break;
                }
            }
        }
        __syncthreads();
    }
    for (uint32_t q = tid; q < J.nstore * KQ; q += nthr) {
        const uint32_t cell = q / KQ, off = q % KQ;
        reinterpret_cast<uint4 *>(x + (J.base + (uint64_t)cell * J.stride) * K)[off] =
            reinterpret_cast<const uint4 *>(smq)[q];
    }
}

// ---------------------------------------------------------------------------
// negacyclic products mod m with Montgomery reduction (R = 2^64)
// ---------------------------------------------------------------------------

// T = hi:lo < m 2^64  ->  T 2^-64 mod m
__device__ __forceinline__ uint64_t redc(uint64_t lo, uint64_t hi, uint64_t m, uint64_t minv) {
    const uint64_t u = lo * minv;
    const uint64_t uhi = __umul64hi(u, m);
    const uint64_t t = hi + uhi + (lo != 0 ? 1u : 0u);
    return t >= m ? t - m : t;
}

constexpr int NP_COLS = 4;     // columns per thread up to K = 1024 (256 threads); K / 256 above
constexpr int NP_GROUP = 16;  // products per 128-bit partial sum: 16 m^2 < 2^128 for m < 2^62

// a b as a 128-bit value (hi:lo) for a, b < 2^63, from four 32x32 -> 64 multiply-adds
__device__ __forceinline__ void mul128(uint64_t a, uint64_t b, uint64_t &lo, uint64_t &hi) {
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint64_t p00 = (uint64_t)a0 * b0;
    const uint64_t t1 = (uint64_t)a0 * b1 + (p00 >> 32);
    const uint64_t t2 = (uint64_t)a1 * b0 + (uint32_t)t1;
    lo = (t2 << 32) | (uint32_t)p00;
    hi = (uint64_t)a1 * b1 + (t1 >> 32) + (t2 >> 32);
}

template <int J, int N, class Fn>
__device__ __forceinline__ void nega_static_for(Fn &&f) {
    if constexpr (J < N) {
        f(std::integral_constant<int, J>{});
        nega_static_for<J + 1, N>(f);
    }
}

// Four columns of products av * bw[c] (both < 2^63) added into column sums
// kept as three accumulators per column: s0 = sum a0 b0 (+ 2^64 w0 wraps),
// s1 = sum a0 b1 + a1 b0 (+ 2^64 w1 wraps), s2 = sum a1 b1 (no wrap within a
// group), with a = a1 2^32 + a0.  Each wrapping sum takes a 64-bit multiply-add
// with its carry-out into an SGPR pair and an add-with-carry into its count;
// four multiply-adds precede their four carry reads (the VALU SGPR-write to
// carry-read hazard needs two wait states).  Registers only (no memory access).
template <int C0, int NC>
__device__ __forceinline__ void nega_mac4(uint64_t (&acc)[NC], uint32_t (&w)[NC], uint32_t a,
                                          const uint32_t (&b)[NC]) {
    uint64_t c0, c1, c2, c3;
    asm("v_mad_u64_u32 %0, %4, %8, %9, %0\n\t"
        "v_mad_u64_u32 %1, %5, %8, %10, %1\n\t"
        "v_mad_u64_u32 %2, %6, %8, %11, %2\n\t"
        "v_mad_u64_u32 %3, %7, %8, %12, %3"
        : "+v"(acc[C0]), "+v"(acc[C0 + 1]), "+v"(acc[C0 + 2]), "+v"(acc[C0 + 3]), "=&s"(c0), "=&s"(c1), "=&s"(c2),
          "=&s"(c3)
        : "v"(a), "v"(b[C0]), "v"(b[C0 + 1]), "v"(b[C0 + 2]), "v"(b[C0 + 3]));
    asm("v_addc_co_u32_e64 %0, %4, %0, 0, %4\n\t"
        "v_addc_co_u32_e64 %1, %5, %1, 0, %5\n\t"
        "v_addc_co_u32_e64 %2, %6, %2, 0, %6\n\t"
        "v_addc_co_u32_e64 %3, %7, %3, 0, %7"
        : "+v"(w[C0]), "+v"(w[C0 + 1]), "+v"(w[C0 + 2]), "+v"(w[C0 + 3]), "+s"(c0), "+s"(c1), "+s"(c2), "+s"(c3));
}

// c_k = sum_i a_i b_{k-i} - sum_{i>k} a_i b_{k-i+K}  (mod m, y^K = -1), times 2^-scale.
// Each thread owns NP_COLS consecutive columns and slides a register window
// over B2 = [b, m - b] (the wrapped terms enter negated, so every product is
// unsigned): the word entering the window is negated when its index wraps.
// Products are summed in 128 bits and reduced (Montgomery, R = 2^64) every
// NP_GROUP terms after the high word is brought below m.
template <int K>
__global__ void __launch_bounds__(256) nega_pointwise_kernel(const uint64_t *__restrict__ a,
                                                             const uint64_t *__restrict__ b, uint64_t *c, uint64_t m,
                                                             uint64_t minv, uint64_t cfac) {
    extern __shared__ uint64_t nega_pw_sm[];  // A (K words) then B (K words)
    uint64_t *A = nega_pw_sm, *B = nega_pw_sm + K;
    const uint64_t i = blockIdx.x;
    const uint32_t tid = threadIdx.x, nthr = blockDim.x;
    for (uint32_t q = tid; q < (uint32_t)K; q += nthr) {
        A[q] = a[i * K + q];
        B[q] = b[i * K + q];
    }
    __syncthreads();
    constexpr int NC = K < NP_COLS ? K : (K > 256 * NP_COLS ? K / 256 : NP_COLS);
    uint64_t res[NC];
    bool have = false;
    const uint32_t k0 = tid * NC;
    if (k0 < (uint32_t)K) {
        have = true;
        const uint64_t m2 = 2 * m;
        uint64_t lo[NC], hi[NC], r[NC], bw[NC];
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
            lo[cc] = hi[cc] = r[cc] = 0;
            bw[cc] = B[k0 + cc];  // window at i = 0: B2[k0 + cc]
        }
        // four-column blocks: partial products in three column accumulators
        uint64_t s0[NC], s1[NC], s2[NC];
        uint32_t w0[NC], w1[NC];
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
            s0[cc] = s1[cc] = s2[cc] = 0;
            w0[cc] = w1[cc] = 0;
        }
        for (uint32_t ii = 0; ii < (uint32_t)K; ++ii) {
            const uint64_t av = A[ii];
            if constexpr (NC % 4 == 0) {
                const uint32_t a0 = (uint32_t)av, a1 = (uint32_t)(av >> 32);
                uint32_t b0[NC], b1[NC];
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) {
                    b0[cc] = (uint32_t)bw[cc];
                    b1[cc] = (uint32_t)(bw[cc] >> 32);
                }
                nega_static_for<0, NC / 4>([&](auto qc) {
                    constexpr int c4 = 4 * decltype(qc)::value;
                    nega_mac4<c4, NC>(s0, w0, a0, b0);
                    nega_mac4<c4, NC>(s1, w1, a0, b1);
                    nega_mac4<c4, NC>(s1, w1, a1, b0);
                });
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) s2[cc] += (uint64_t)a1 * b1[cc];  // < 16 2^60, no wrap
            } else {
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) {
                    uint64_t pl, ph;
                    mul128(av, bw[cc], pl, ph);
                    lo[cc] += pl;
                    hi[cc] += ph + (lo[cc] < pl ? 1u : 0u);
                }
            }
            if ((ii & (NP_GROUP - 1)) == NP_GROUP - 1 || ii + 1 == (uint32_t)K) {
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) {
                    if constexpr (NC % 4 == 0) {
                        // sum = s0 + 2^64 w0 + 2^32 (s1 + 2^64 w1) + 2^64 s2
                        const uint64_t t = s1[cc] << 32;
                        lo[cc] = s0[cc] + t;
                        hi[cc] = (uint64_t)w0[cc] + (s1[cc] >> 32) + ((uint64_t)w1[cc] << 32) + s2[cc] +
                                 (lo[cc] < t ? 1u : 0u);
                        s0[cc] = s1[cc] = s2[cc] = 0;
                        w0[cc] = w1[cc] = 0;
                    }
                    uint64_t h = hi[cc];  // < 16 m^2 / 2^64 < 4 m
                    h = h >= m2 ? h - m2 : h;
                    h = h >= m ? h - m : h;
                    r[cc] = madd(r[cc], redc(lo[cc], h, m, minv), m);
                    lo[cc] = hi[cc] = 0;
                }
            }
#pragma unroll
            for (int cc = NC - 1; cc > 0; --cc) bw[cc] = bw[cc - 1];
            // column k0 at step ii + 1 needs B2[(k0 - ii - 1) mod 2K]
            const uint64_t bv = B[(k0 - ii - 1u) & (K - 1u)];
            bw[0] = ii + 1u <= k0 ? bv : m - bv;
        }
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
            // r = (sum) 2^-64; times cfac = 2^128 2^-scale, reduced once more
            uint64_t pl, ph;
            mul128(r[cc], cfac, pl, ph);
            res[cc] = redc(pl, ph, m, minv);
        }
    }
    __syncthreads();  // c may alias a or b
    if (have) {
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) c[i * K + k0 + cc] = res[cc];
    }
}

__global__ void nega_pack_kernel(const uint64_t *__restrict__ coef, uint64_t len, uint64_t *__restrict__ x,
                                 uint64_t pieces, uint32_t K) {
    const uint64_t total = pieces * K, half = K / 2;
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < total;
         q += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t p = q / K, j = q % K;
        const uint64_t src = p * half + j;
        x[q] = (j < half && src < len) ? coef[src] : 0u;
    }
}

__global__ void nega_unpack_kernel(const uint64_t *__restrict__ x, uint64_t pieces, uint64_t *__restrict__ out,
                                   uint64_t out_len, uint32_t K, uint64_t m) {
    const uint64_t half = K / 2;
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < out_len;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t p = t / half, j = t % half;
        uint64_t v = p < pieces ? x[p * K + j] : 0u;
        if (p >= 1 && p - 1 < pieces) v = madd(v, x[(p - 1) * K + j + half], m);
        out[t] = v;
    }
}

template <int S, int R>
hipError_t nega_leaf_launch(uint64_t m, uint32_t nwaves, uint32_t njobs, uint32_t lds_cells, const Job *jobs,
                            uint32_t job_offset, const LeafProg *progs, const LeafStep *steps, const LeafOp *ops,
                            uint64_t *x, uint32_t ord_mask, hipStream_t st) {
    constexpr int K = S * R;
    const size_t lds = (size_t)lds_cells * K * 8;
    if (lds > kLdsBudget) return hipErrorInvalidValue;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&nega_leaf_kernel<S, R>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const uint32_t per = kMaxGridX / (64 * nwaves);
    for (uint32_t j0 = 0; j0 < njobs; j0 += per) {
        const uint32_t nb = njobs - j0 < per ? njobs - j0 : per;
        hipLaunchKernelGGL((nega_leaf_kernel<S, R>), dim3(nb), dim3(64 * nwaves), lds, st, jobs, progs, steps, ops, x,
                           m, ord_mask, job_offset + j0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int K>
hipError_t nega_pw_launch(uint64_t m, uint64_t n, const uint64_t *a, const uint64_t *b, uint64_t *c,
                          uint32_t scale_log2, hipStream_t st) {
    // host constants: minv = -m^-1 mod 2^64, cfac = 2^128 * 2^-scale mod m
    uint64_t inv = 1;
    for (int it = 0; it < 7; ++it) inv *= 2 - m * inv;  // Newton: m * inv = 1 mod 2^64
    const uint64_t minv = 0 - inv;
    unsigned __int128 r = ((unsigned __int128)1 << 64) % m;
    r = (r * r) % m;  // 2^128 mod m
    const uint64_t inv2 = (m + 1) / 2;
    for (uint32_t t = 0; t < scale_log2; ++t) r = (r * inv2) % m;
    const uint64_t cfac = (uint64_t)r;
    constexpr int NC = K < NP_COLS ? K : (K > 256 * NP_COLS ? K / 256 : NP_COLS);
    uint32_t thr = (K + NC - 1) / NC;
    thr = thr < 64 ? 64 : (thr > 256 ? 256 : thr);
    thr = (thr + 63) / 64 * 64;
    if ((uint32_t)K > thr * NC) return hipErrorInvalidValue;
    const size_t lds = 2ull * K * sizeof(uint64_t);
    static bool attr = false;
    if (!attr && lds >= 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&nega_pointwise_kernel<K>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const uint64_t per = kMaxGridX / thr;
    for (uint64_t i0 = 0; i0 < n; i0 += per) {
        const uint64_t nb = n - i0 < per ? n - i0 : per;
        hipLaunchKernelGGL((nega_pointwise_kernel<K>), dim3((uint32_t)nb), dim3(thr), lds, st, a + i0 * K, b + i0 * K,
                           c + i0 * K, m, minv, cfac);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

#define TFT_NEGA_DISPATCH(K, FN, ...)              \
    switch (K) {                                   \
        case 2: return FN<2, 1>(__VA_ARGS__);      \
        case 4: return FN<4, 1>(__VA_ARGS__);      \
        case 8: return FN<8, 1>(__VA_ARGS__);      \
        case 16: return FN<16, 1>(__VA_ARGS__);    \
        case 32: return FN<32, 1>(__VA_ARGS__);    \
        case 64: return FN<64, 1>(__VA_ARGS__);    \
        case 128: return FN<64, 2>(__VA_ARGS__);   \
        case 256: return FN<64, 4>(__VA_ARGS__);   \
        case 512: return FN<64, 8>(__VA_ARGS__);   \
        case 1024: return FN<64, 16>(__VA_ARGS__); \
        case 2048: return FN<64, 32>(__VA_ARGS__); \
        case 4096: return FN<64, 64>(__VA_ARGS__); \
        default: return hipErrorInvalidValue;      \
    }

hipError_t launch_nega_leaf(uint32_t K, uint64_t m, uint32_t nwaves, uint32_t njobs, uint32_t lds_cells,
                            const Job *jobs, uint32_t job_offset, const LeafProg *progs, const LeafStep *steps,
                            const LeafOp *ops, uint64_t *x, uint32_t ord_mask, hipStream_t st) {
    if (njobs == 0) return hipSuccess;
    TFT_NEGA_DISPATCH(K, nega_leaf_launch, m, nwaves, njobs, lds_cells, jobs, job_offset, progs, steps, ops, x,
                      ord_mask, st)
}

hipError_t launch_nega_pointwise(uint32_t K, uint64_t m, uint64_t n, const uint64_t *a, const uint64_t *b,
                                 uint64_t *c, uint32_t scale_log2, hipStream_t st) {
    if (n == 0) return hipSuccess;
    switch (K) {
        case 2: return nega_pw_launch<2>(m, n, a, b, c, scale_log2, st);
        case 4: return nega_pw_launch<4>(m, n, a, b, c, scale_log2, st);
        case 8: return nega_pw_launch<8>(m, n, a, b, c, scale_log2, st);
        case 16: return nega_pw_launch<16>(m, n, a, b, c, scale_log2, st);
        case 32: return nega_pw_launch<32>(m, n, a, b, c, scale_log2, st);
        case 64: return nega_pw_launch<64>(m, n, a, b, c, scale_log2, st);
        case 128: return nega_pw_launch<128>(m, n, a, b, c, scale_log2, st);
        case 256: return nega_pw_launch<256>(m, n, a, b, c, scale_log2, st);
        case 512: return nega_pw_launch<512>(m, n, a, b, c, scale_log2, st);
        case 1024: return nega_pw_launch<1024>(m, n, a, b, c, scale_log2, st);
        case 2048: return nega_pw_launch<2048>(m, n, a, b, c, scale_log2, st);
        case 4096: return nega_pw_launch<4096>(m, n, a, b, c, scale_log2, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_nega_pack(uint32_t K, const uint64_t *coef, uint64_t len, uint64_t *x, uint64_t pieces,
                            hipStream_t st) {
    if (pieces == 0) return hipSuccess;
    const uint64_t total = pieces * K;
    uint32_t blocks = (uint32_t)((total + 255) / 256);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(nega_pack_kernel, dim3(blocks), dim3(256), 0, st, coef, len, x, pieces, K);
    return hipGetLastError();
}

hipError_t launch_nega_unpack(uint32_t K, uint64_t m, const uint64_t *x, uint64_t pieces, uint64_t *out,
                              uint64_t out_len, hipStream_t st) {
    if (out_len == 0) return hipSuccess;
    uint32_t blocks = (uint32_t)((out_len + 255) / 256);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(nega_unpack_kernel, dim3(blocks), dim3(256), 0, st, x, pieces, out, out_len, K, m);
    return hipGetLastError();
}

}  // namespace tft
