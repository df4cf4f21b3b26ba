// Leaf executor and pointwise products for R = Z/pZ, the word-size prime of
// the small-coefficient case (Sect. 6): the jobs, programs and base cases of
// Alg. 1 and Alg. 2 that the host planner builds for every ring, on residues
// of one 32-bit word.
//
// Sect. 6 notes that column sub-transforms touch words a large power of two
// apart, and that the cure is to transpose the matrix while they run.  Here a
// workgroup takes `pack` jobs of a pass at once, the pass's jobs sorted by
// their first cell: for a column pass (stride > 1) the jobs are adjacent
// columns, and element (p, r) of the pack is read with p varying fastest, so
// a wave reads consecutive words of one row and the tile lands in LDS as the
// transposed block; row passes (stride 1) read along the row.  Each job keeps
// its cells in LDS at pitch slot + 1 words, so the lanes that run the same
// base case on adjacent jobs hit different banks.
//
// Twiddles: a base case's exponent is s 2^alog + b (s the job's twist).  The
// factor theta^b is the op's entry in a table the host builds with the plan
// (theta^-b for the inverse butterfly of Alg. 2); theta^(s 2^alog) is computed
// once per job and pack into LDS.  One Montgomery product joins them.
#include <hip/hip_runtime.h>

#include "desc.hpp"
#include "kernels.hpp"
#include "prime.hpp"

namespace tft {

namespace {

constexpr uint32_t kZpThreads = 256;
constexpr uint32_t kZpLdsWords = 40960;  // 160 KB
constexpr uint32_t kDescWords = 8;      // base lo, base hi, stride lo, stride hi, nload, nstore, prog, s

__device__ __forceinline__ void zp_base_case(uint32_t *c, uint32_t code, uint32_t i0, uint32_t i1, uint32_t zm) {
    using namespace zp;
    const uint32_t a = c[i0];
    switch (code) {
        case OP_T22: {  // (x0 + x1, zeta (x0 - x1))
            const uint32_t b = c[i1];
            c[i0] = add(a, b);
            c[i1] = mont(sub(a, b), zm);
            break;
        }
        case OP_T21:  // x1 = zeta x0
            c[i1] = mont(a, zm);
            break;
        case OP_T12:  // x0 = x0 + x1
            c[i0] = add(a, c[i1]);
            break;
        case OP_I2: {  // (x0 + x1 / zeta, x0 - x1 / zeta); zm holds zeta^-1
            const uint32_t t = mont(c[i1], zm);
            c[i0] = add(a, t);
            c[i1] = sub(a, t);
            break;
        }
        case OP_I1F1Z2: {  // (2 x0 - x1, zeta (x0 - x1))
            const uint32_t b = c[i1];
            c[i0] = sub(add(a, a), b);
            c[i1] = mont(sub(a, b), zm);
            break;
        }
        case OP_I1F1Z1:  // (2 x0, zeta x0)
            c[i1] = mont(a, zm);
            c[i0] = add(a, a);
            break;
        case OP_I1F0Z2:  // x0 = 2 x0 - x1
            c[i0] = sub(add(a, a), c[i1]);
            break;
        case OP_I1F0Z1:  // x0 = 2 x0
            c[i0] = add(a, a);
            break;
        case OP_I0Z2:  // x0 = (x0 + x1) / 2
            c[i0] = half(add(a, c[i1]));
            break;
        case OP_I0Z1:  // x0 = x0 / 2
            c[i0] = half(a);
            break;
        default: break;
    }
}

// One base case (op j of a step) of job p: its cells at c, its twist table at zt.
__device__ __forceinline__ void zp_op(uint32_t *c, const uint32_t *zt, uint32_t zw, const LeafOp &o, uint32_t tw) {
    const uint32_t code = o.w0 & 15u;
    const uint32_t i0 = (o.w0 >> 4) & 16383u, i1 = (o.w0 >> 18) & 16383u;
    const uint32_t alog = op_alog(o);
    const uint32_t zm = zp::mont(zt[(code == OP_I2 ? zw : 0u) + alog], tw);
    zp_base_case(c, code, i0, i1, zm);
}

// floor(k / d) for k < 2^24 and 1 <= d < 2^24 (a float estimate, then one correction)
__device__ __forceinline__ uint32_t div_small(uint32_t k, uint32_t d, float rd) {
    uint32_t q = (uint32_t)((float)k * rd);
    if (q * d > k) --q;
    else if ((q + 1u) * d <= k) ++q;
    return q;
}

// A workgroup runs jobs [first, first + count) of a pass, `pack` = 2^pack_log2
// jobs of 2^slot_log2 cells at most; zw = twist entries per job (alog < zw).
__global__ void __launch_bounds__(kZpThreads) zp_leaf_kernel(const Job *__restrict__ jobs,
                                                             const LeafProg *__restrict__ progs,
                                                             const LeafStep *__restrict__ steps,
                                                             const LeafOp *__restrict__ ops,
                                                             const uint32_t *__restrict__ optw,
                                                             uint32_t *__restrict__ x, uint32_t job_begin,
                                                             uint32_t njobs, uint32_t pack_log2, uint32_t slot_log2,
                                                             uint32_t zw) {
    extern __shared__ uint32_t sm[];
    const uint32_t tid = threadIdx.x;
    const uint32_t pack = 1u << pack_log2, slot = 1u << slot_log2, pitch = slot + 1u;
    const uint32_t first = blockIdx.x * pack;
    const uint32_t count = njobs - first < pack ? njobs - first : pack;
    jobs += job_begin + first;
    uint32_t *dsc = sm;                          // kDescWords per job
    uint32_t *ztab = dsc + kDescWords * pack;    // 2 zw per job: theta^(s 2^a), theta^(-s 2^a), Montgomery form
    uint32_t *dat = ztab + 2u * zw * pack;       // job p's cells at p * pitch

    for (uint32_t p = tid; p < count; p += kZpThreads) {
        const Job J = jobs[p];
        uint32_t *d = dsc + kDescWords * p;
        d[0] = (uint32_t)J.base;
        d[1] = (uint32_t)(J.base >> 32);
        d[2] = (uint32_t)J.stride;
        d[3] = (uint32_t)(J.stride >> 32);
        d[4] = J.nload;
        d[5] = J.nstore;
        d[6] = J.prog;
        d[7] = J.s;
    }
    for (uint32_t q = tid; q < count * zw; q += kZpThreads) {
        const uint32_t p = q / zw, a = q - p * zw;
        const uint64_t e = ((uint64_t)jobs[p].s << a) & (zp::ORD - 1u);
        ztab[2u * zw * p + a] = zp::theta_pow_m(e);
        ztab[2u * zw * p + zw + a] = zp::theta_pow_m(zp::ORD - e);
    }
    __syncthreads();

    // element e of the pack: (job, cell); rows read along the row, columns across jobs
    const bool rows = dsc[2] == 1u && dsc[3] == 0u;
    const uint32_t E = rows ? count << slot_log2 : pack << slot_log2;
    auto elem = [&](uint32_t e, uint32_t &p, uint32_t &r) {
        if (rows) {
            p = e >> slot_log2;
            r = e & (slot - 1u);
        } else {
            p = e & (pack - 1u);
            r = e >> pack_log2;
        }
    };
    auto gaddr = [&](uint32_t p, uint32_t r) {
        const uint32_t *d = dsc + kDescWords * p;
        const uint64_t base = (uint64_t)d[1] << 32 | d[0], stride = (uint64_t)d[3] << 32 | d[2];
        return base + (uint64_t)r * stride;
    };
    for (uint32_t e = tid; e < E; e += kZpThreads) {
        uint32_t p, r;
        elem(e, p, r);
        if (p < count && r < dsc[kDescWords * p + 4]) dat[p * pitch + r] = x[gaddr(p, r)];
    }
    __syncthreads();

    // the programs, step by step; all jobs of one program: items (job, op) with
    // the op varying fastest; otherwise job after job
    uint32_t same = 1u;
    for (uint32_t p = 1; p < count; ++p) same &= dsc[kDescWords * p + 6] == dsc[6] ? 1u : 0u;
    if (same) {
        const LeafProg P = progs[dsc[6]];
        for (uint32_t st = 0; st < P.step_count; ++st) {
            const LeafStep LS = steps[P.step_begin + st];
            const uint32_t oc = LS.op_count;
            const float rd = 1.0f / (float)(oc ? oc : 1u);
            const bool p2 = (oc & (oc - 1u)) == 0u;
            uint32_t ol = 0;
            while ((1u << ol) < oc) ++ol;
            for (uint32_t k = tid; k < count * oc; k += kZpThreads) {
                const uint32_t p = p2 ? k >> ol : div_small(k, oc, rd);
                const uint32_t j = k - p * oc;
                zp_op(dat + p * pitch, ztab + 2u * zw * p, zw, ops[LS.op_begin + j], optw[LS.op_begin + j]);
            }
            __syncthreads();
        }
    } else {
        for (uint32_t p = 0; p < count; ++p) {
            const LeafProg P = progs[dsc[kDescWords * p + 6]];
            for (uint32_t st = 0; st < P.step_count; ++st) {
                const LeafStep LS = steps[P.step_begin + st];
                for (uint32_t j = tid; j < LS.op_count; j += kZpThreads)
                    zp_op(dat + p * pitch, ztab + 2u * zw * p, zw, ops[LS.op_begin + j], optw[LS.op_begin + j]);
                __syncthreads();
            }
        }
    }

    for (uint32_t e = tid; e < E; e += kZpThreads) {
        uint32_t p, r;
        elem(e, p, r);
        if (p < count && r < dsc[kDescWords * p + 5]) x[gaddr(p, r)] = dat[p * pitch + r];
    }
}

// c_i = a_i b_i 2^-s: k = 2^-s R^2 mod p (two Montgomery products)
__global__ void __launch_bounds__(256) zp_pointwise_kernel(const uint32_t *__restrict__ a,
                                                           const uint32_t *__restrict__ b, uint32_t *c, uint64_t n,
                                                           uint32_t k) {
    const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    if (i < n) c[i] = zp::mont(zp::mont(a[i], b[i]), k);
}

}  // namespace

uint32_t zp_leaf_pack_log2(uint32_t njobs, uint32_t slot_log2, uint32_t zw) {
    const uint32_t per = kDescWords + 2u * zw + (1u << slot_log2) + 1u;
    uint32_t pl = 0;
    while ((2u << pl) * per <= kZpLdsWords && (2u << pl) <= 1024u) ++pl;
    // keep at least two workgroups per compute unit when the pass has the jobs
    while (pl > 0 && (njobs >> pl) < 512u) --pl;
    return pl;
}

hipError_t launch_zp_leaf(uint32_t njobs, uint32_t max_len, const Job *jobs, uint32_t job_begin,
                          const LeafProg *progs, const LeafStep *steps, const LeafOp *ops, const uint32_t *optw,
                          uint32_t *x, uint32_t zw, hipStream_t st) {
    if (njobs == 0) return hipSuccess;
    uint32_t sl = 0;
    while ((1u << sl) < max_len) ++sl;
    if ((1u << sl) != max_len || zw == 0 || zw > 16) return hipErrorInvalidValue;
    const uint32_t pl = zp_leaf_pack_log2(njobs, sl, zw);
    const uint32_t pack = 1u << pl;
    const size_t words = (size_t)pack * (kDescWords + 2u * zw + max_len + 1u);
    if (words > kZpLdsWords) return hipErrorInvalidValue;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&zp_leaf_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kZpLdsWords * 4u));
        if (e != hipSuccess) return e;
        attr = true;
    }
    const uint32_t grid = (njobs + pack - 1u) >> pl;
    hipLaunchKernelGGL(zp_leaf_kernel, dim3(grid), dim3(kZpThreads), words * 4u, st, jobs, progs, steps, ops, optw, x,
                       job_begin, njobs, pl, sl, zw);
    return hipGetLastError();
}

hipError_t launch_zp_pointwise(uint64_t n, const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t scale_log2,
                               hipStream_t st) {
    if (n == 0) return hipSuccess;
    const uint32_t inv = zp::from_mont(zp::pow_m(zp::to_mont((zp::P + 1u) / 2u), scale_log2));  // 2^-s
    const uint32_t k = zp::to_mont(zp::to_mont(inv));
    hipLaunchKernelGGL(zp_pointwise_kernel, dim3((uint32_t)((n + 255u) / 256u)), dim3(256), 0, st, a, b, c, n, k);
    return hipGetLastError();
}

}  // namespace tft
