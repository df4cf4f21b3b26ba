// Leaf executor of the cache-friendly TFT/ITFT (Alg. 1, Alg. 2) in
// R = Z/(2^N+1): kernels and launch helpers shared by the translation units
// that instantiate them for the two global cell layouts (plain: limbs in
// order; transposed: the LDS order of fermat_dev.hpp, used inside products).
#pragma once
#include <hip/hip_runtime.h>

#include "desc.hpp"
#include "fermat_dev.hpp"
#include "kernels.hpp"

namespace tft {

namespace {

constexpr uint32_t kLdsBudget = 160u * 1024u;
// work-items per grid dimension of one launch (the dispatch packet holds 32-bit sizes)
constexpr uint32_t kMaxGridX = 0xFFFFFFFFu;
constexpr uint32_t kLeafStaticLds = 0u;  // no static LDS in fermat_leaf_kernel

// Copy leaf cells [0, n) between the global array (cell-contiguous limbs) and
// LDS (cells ESZ dwords apart, limb k at F::addr(k)).  With one element per
// wave the 64 lanes of a wave take 64 different LDS columns (limbs l C ..
// l C + 3 of the cell for lane l), so every LDS access of the copy is
// conflict-free; each thread keeps CB global accesses in flight before
// touching LDS.
constexpr int CB = 8;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <class F, bool IN, bool TR>
__device__ __forceinline__ void copy_cells(uint32_t *sm, uint32_t *x, const Job &J, uint32_t n, uint32_t tid,
                                           uint32_t nthr) {
    constexpr int W = F::W, C = F::C;
    if constexpr (TR || F::S < 64) {
        // the global cell has the LDS order: a straight copy
        if constexpr (W % 4 == 0) {
            constexpr uint32_t WQ = W / 4;
            const uint32_t total = n * WQ;
            for (uint32_t q0 = tid; q0 < total; q0 += nthr * CB) {
                u32x4 v[CB];
                if (IN) {
#pragma unroll
                    for (int b = 0; b < CB; ++b) {
                        const uint32_t q = q0 + b * nthr;
                        if (q < total) {
                            const uint32_t cell = q / WQ, off = q % WQ;
                            v[b] = reinterpret_cast<const u32x4 *>(x + (J.base + (uint64_t)cell * J.stride) * W)[off];
                        }
                    }
#pragma unroll
                    for (int b = 0; b < CB; ++b) {
                        const uint32_t q = q0 + b * nthr;
                        if (q < total) reinterpret_cast<u32x4 *>(sm + (q / WQ) * F::ESZ)[q % WQ] = v[b];
                    }
                } else {
#pragma unroll
                    for (int b = 0; b < CB; ++b) {
                        const uint32_t q = q0 + b * nthr;
                        if (q < total) v[b] = reinterpret_cast<const u32x4 *>(sm + (q / WQ) * F::ESZ)[q % WQ];
                    }
#pragma unroll
                    for (int b = 0; b < CB; ++b) {
                        const uint32_t q = q0 + b * nthr;
                        if (q < total) {
                            const uint32_t cell = q / WQ, off = q % WQ;
                            reinterpret_cast<u32x4 *>(x + (J.base + (uint64_t)cell * J.stride) * W)[off] = v[b];
                        }
                    }
                }
            }
        } else {
            const uint32_t total = n * W;
            for (uint32_t q = tid; q < total; q += nthr) {
                const uint32_t cell = q / W, off = q % W;
                uint32_t *g = x + (J.base + (uint64_t)cell * J.stride) * W + off;
                if (IN)
                    sm[cell * F::ESZ + off] = *g;
                else
                    *g = sm[cell * F::ESZ + off];
            }
        }
    } else if constexpr (C >= 4) {
        constexpr uint32_t WQ = W / 4, CQ = C / 4;
        const uint32_t total = n * WQ;
        for (uint32_t q0 = tid; q0 < total; q0 += nthr * CB) {
            uint4 v[CB];
            uint32_t *g[CB];
            uint32_t *s[CB];
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                const uint32_t q = q0 + b * nthr;
                const uint32_t cell = q / WQ, r = q % WQ, l = r % 64u, m = r / 64u;
                g[b] = x + (J.base + (uint64_t)cell * J.stride) * W + (l * CQ + m) * 4u;
                s[b] = sm + cell * F::ESZ + 4u * m * 64u + l;
            }
            if (IN) {
#pragma unroll
                for (int b = 0; b < CB; ++b)
                    if (q0 + b * nthr < total) v[b] = *reinterpret_cast<const uint4 *>(g[b]);
#pragma unroll
                for (int b = 0; b < CB; ++b)
                    if (q0 + b * nthr < total) {
                        s[b][0] = v[b].x;
                        s[b][64] = v[b].y;
                        s[b][128] = v[b].z;
                        s[b][192] = v[b].w;
                    }
            } else {
#pragma unroll
                for (int b = 0; b < CB; ++b)
                    if (q0 + b * nthr < total) v[b] = make_uint4(s[b][0], s[b][64], s[b][128], s[b][192]);
#pragma unroll
                for (int b = 0; b < CB; ++b)
                    if (q0 + b * nthr < total) *reinterpret_cast<uint4 *>(g[b]) = v[b];
            }
        }
    } else if constexpr (F::S == 64) {
        const uint32_t total = n * W;
        for (uint32_t q = tid; q < total; q += nthr) {
            const uint32_t cell = q / W, r = q % W, l = r % 64u, j = r / 64u;
            uint32_t *g = x + (J.base + (uint64_t)cell * J.stride) * W + l * C + j;
            uint32_t *t = sm + cell * F::ESZ + j * 64u + l;
            if (IN)
                *t = *g;
            else
                *g = *t;
        }
    }
}

// Base-case sets a leaf kernel is compiled for.  Keeping the rare boundary
// cases out of the hot kernels keeps their register allocation within 256
// VGPRs (no spills) for the largest elements.
enum LeafSet : int { SET_TFT = 0, SET_ITFT = 1, SET_ALL = 2 };
constexpr uint32_t kTftOps = (1u << OP_T22) | (1u << OP_T21) | (1u << OP_T12);
constexpr uint32_t kItftOps = (1u << OP_I2) | (1u << OP_I1F1Z2) | (1u << OP_I1F0Z2) | (1u << OP_I1F0Z1);

template <int V>
constexpr bool set_has(uint32_t code) {
    return V == SET_ALL || (V == SET_TFT ? ((kTftOps >> code) & 1u) : ((kItftOps >> code) & 1u));
}

template <int S, int C, int V, bool TR>
__device__ __forceinline__ void leaf_body(const Job *__restrict__ jobs, const LeafProg *__restrict__ progs,
                                          const LeafStep *__restrict__ steps, const LeafOp *__restrict__ ops,
                                          uint32_t *__restrict__ x, uint64_t cap, uint32_t ord_mask,
                                          uint32_t lds_cells, uint32_t job_offset) {
    using F = FChunk<S, C>;
    constexpr int W = F::W;
    constexpr uint32_t G = 64 / S;
    extern __shared__ uint32_t sm[];
    uint32_t *stop = sm + (size_t)lds_cells * F::ESZ;
    const Job J = jobs[job_offset + blockIdx.x];
    const LeafProg P = progs[J.prog];
    const uint32_t tid = threadIdx.x, nthr = blockDim.x;

    copy_cells<F, true, TR>(sm, x, J, J.nload, tid, nthr);
    for (uint32_t t = tid; t < J.nload; t += nthr) stop[t] = x[cap * W + J.base + (uint64_t)t * J.stride];
    __syncthreads();

    const FermatOps<F> B;
    const uint32_t wave = tid >> 6, nwaves = nthr >> 6;
    const uint32_t g = B.lane / S;
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
                uint32_t *x0 = sm + i0 * F::ESZ, *x1 = sm + i1 * F::ESZ;
                uint32_t *t0 = stop + i0, *t1 = stop + i1;
                switch (code) {
                    case OP_T22:
                        if constexpr (set_has<V>(OP_T22)) B.t22(x0, x1, t0, t1, e);
                        break;
                    case OP_T21:
                        if constexpr (set_has<V>(OP_T21)) B.t21(x0, x1, t0, t1, e);
                        break;
                    case OP_T12:
                        if constexpr (set_has<V>(OP_T12)) B.add2(x0, x1, t0, t1);
                        break;
                    case OP_I2:
                        if constexpr (set_has<V>(OP_I2)) B.i2(x0, x1, t0, t1, (0u - e) & ord_mask);
                        break;
                    case OP_I1F1Z2:
                        if constexpr (set_has<V>(OP_I1F1Z2)) B.i1f1(x0, x1, t0, t1, e, true);
                        break;
                    case OP_I1F1Z1:
                        if constexpr (set_has<V>(OP_I1F1Z1)) B.i1f1(x0, x1, t0, t1, e, false);
                        break;
                    case OP_I1F0Z2:
                        if constexpr (set_has<V>(OP_I1F0Z2)) B.dbl_sub(x0, x1, t0, t1);
                        break;
                    case OP_I1F0Z1:
                        if constexpr (set_has<V>(OP_I1F0Z1)) B.dbl_sub(x0, nullptr, t0, nullptr);
                        break;
                    case OP_I0Z2:
                        if constexpr (set_has<V>(OP_I0Z2)) {
                            B.add2(x0, x1, t0, t1);
                            B.scale(x0, t0, ord_mask);  // 2^(2N-1) = 1/2
                        }
                        break;
                    case OP_I0Z1:
                        if constexpr (set_has<V>(OP_I0Z1)) B.scale(x0, t0, ord_mask);
                        break;
                    default: break;
                }
            }
        }
        __syncthreads();
    }

    copy_cells<F, false, TR>(sm, x, J, J.nstore, tid, nthr);
    for (uint32_t t = tid; t < J.nstore; t += nthr) x[cap * W + J.base + (uint64_t)t * J.stride] = stop[t];
}

template <int S, int C, int V, bool TR>
__global__ void __launch_bounds__(512) fermat_leaf_kernel(const Job *__restrict__ jobs,
                                                           const LeafProg *__restrict__ progs,
                                                           const LeafStep *__restrict__ steps,
                                                           const LeafOp *__restrict__ ops, uint32_t *__restrict__ x,
                                                           uint64_t cap, uint32_t ord_mask, uint32_t lds_cells,
                                                           uint32_t job_offset) {
    leaf_body<S, C, V, TR>(jobs, progs, steps, ops, x, cap, ord_mask, lds_cells, job_offset);
}

template <int S, int C, int V, bool TR>
hipError_t leaf_launch_set(uint32_t nwaves, uint32_t njobs, uint32_t lds_cells, const Job *jobs, uint32_t job_offset,
                           const LeafProg *progs, const LeafStep *steps, const LeafOp *ops, uint32_t *x, uint64_t cap,
                           uint32_t ord_mask, hipStream_t st) {
    const size_t lds = (size_t)lds_cells * (FChunk<S, C>::ESZ + 1) * 4;
    if (lds > kLdsBudget - kLeafStaticLds) return hipErrorInvalidValue;
    auto kern = &fermat_leaf_kernel<S, C, V, TR>;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(kLdsBudget - kLeafStaticLds));
        if (e != hipSuccess) return e;
        attr = true;
    }
    // a launch covers at most 2^32 - 1 work-items per grid dimension
    const uint32_t per = kMaxGridX / (64 * nwaves);
    for (uint32_t j0 = 0; j0 < njobs; j0 += per) {
        const uint32_t nb = njobs - j0 < per ? njobs - j0 : per;
        hipLaunchKernelGGL(kern, dim3(nb), dim3(64 * nwaves), lds, st, jobs, progs, steps, ops, x, cap, ord_mask,
                           lds_cells, job_offset + j0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <bool TR>
struct LeafLaunch {
    template <int S, int C>
    static hipError_t run(uint32_t nwaves, uint32_t njobs, uint32_t lds_cells, const Job *jobs, uint32_t job_offset,
                       const LeafProg *progs, const LeafStep *steps, const LeafOp *ops, uint32_t *x, uint64_t cap,
                       uint32_t ord_mask, uint32_t opmask, hipStream_t st) {
    if ((opmask & ~kTftOps) == 0u)
        return leaf_launch_set<S, C, SET_TFT, TR>(nwaves, njobs, lds_cells, jobs, job_offset, progs, steps, ops, x, cap,
                                              ord_mask, st);
    if ((opmask & ~kItftOps) == 0u)
        return leaf_launch_set<S, C, SET_ITFT, TR>(nwaves, njobs, lds_cells, jobs, job_offset, progs, steps, ops, x, cap,
                                               ord_mask, st);
    return leaf_launch_set<S, C, SET_ALL, TR>(nwaves, njobs, lds_cells, jobs, job_offset, progs, steps, ops, x, cap,
                                          ord_mask, st);
}
};

}  // namespace

#define TFT_FERMAT_DISPATCH(W, FN, ...)                      \
    switch (W) {                                             \
        case 1: return FN<1, 1>(__VA_ARGS__);                \
        case 2: return FN<2, 1>(__VA_ARGS__);                \
        case 4: return FN<4, 1>(__VA_ARGS__);                \
        case 8: return FN<8, 1>(__VA_ARGS__);                \
        case 16: return FN<16, 1>(__VA_ARGS__);              \
        case 32: return FN<32, 1>(__VA_ARGS__);              \
        case 64: return FN<64, 1>(__VA_ARGS__);              \
        case 128: return FN<64, 2>(__VA_ARGS__);             \
        case 256: return FN<64, 4>(__VA_ARGS__);             \
        case 512: return FN<64, 8>(__VA_ARGS__);             \
        case 1024: return FN<64, 16>(__VA_ARGS__);           \
        case 2048: return FN<64, 32>(__VA_ARGS__);           \
        case 4096: return FN<64, 64>(__VA_ARGS__);           \
        default: return hipErrorInvalidValue;                \
    }


}  // namespace tft
