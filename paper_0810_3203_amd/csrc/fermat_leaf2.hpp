// Persistent leaf executor of the cache-friendly TFT/ITFT (Alg. 1, Alg. 2) in
// R = Z/(2^N+1) for one element per wavefront: W = 64 C limbs, C = 4 .. 32.
//
// Every base case of a leaf program (the L = 2 cases of Alg. 1 and Alg. 2)
// runs on one wave: lane l holds limbs [l C, (l+1) C) of an element in
// registers.  The differences from the first executor (fermat_leaf.hpp):
//   * carries and borrows between lanes are resolved by a lookahead over the
//     64 lanes (generate / propagate ballots, one 64-bit addition) instead of
//     a lane-by-lane ripple; the common case costs one limb operation;
//   * the part of a rotation that wraps past 2^N is selected with one
//     and-or per limb from a per-lane and a wave-uniform mask;
//   * rotated LDS reads choose between two non-negative element bases: every
//     cell lies at least one element above the start of the LDS allocation
//     (the first element-sized block holds the top words), so no address is
//     ever formed below the allocation;
//   * a workgroup runs many jobs in turn: while the butterflies of one job run
//     in LDS, the cells of its next job are already being loaded into
//     registers, and the outputs of a job leave LDS in the same sweep that
//     stores the next job's inputs, so copies overlap compute within a CU.
// All device functions are inlined: LDS is reached only through ds_
// instructions on the kernel's own allocation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "desc.hpp"
#include "fermat_leaf2_ops.hpp"
#include "kernels.hpp"
#include "leaf2_addr.hpp"


namespace tft {
namespace lf2 {

template <int C, bool TR>
struct QuadMap {
    static constexpr uint32_t W = 64u * C, K = quad_cells_per_sweep(C);
    uint32_t c0;    // first cell of the thread
    uint32_t loff;  // LDS dword offset of the thread's quad inside its cell
    uint32_t goff;  // dword offset of the thread's quad inside a global cell
    TFT_DINL explicit QuadMap(uint32_t tid)
        : c0(quad_c0(C, tid)), loff(quad_loff(C, TR, tid)), goff(quad_goff(C, TR, tid)) {}
    // dword index (from x) of the thread's quad i of job J
    TFT_DINL uint64_t global(const Job &J, int i) const {
        return (J.base + (uint64_t)(c0 + (uint32_t)i * K) * J.stride) * W + goff;
    }
    TFT_DINL uint32_t lds(int i) const { return cell_base(W, c0 + (uint32_t)i * K) + loff; }
    TFT_DINL bool valid(uint32_t ncells, int i) const { return c0 + (uint32_t)i * K < ncells; }
};

template <bool TR>
TFT_DINL void lds_put_quad(uint32_t *sm, uint32_t a, u32x4 v) {
    if constexpr (TR) {
        *reinterpret_cast<u32x4 *>(sm + a) = v;
    } else {
        constexpr uint32_t d = quad_lds_step(false);
        sm[a] = v.x;
        sm[a + d] = v.y;
        sm[a + 2 * d] = v.z;
        sm[a + 3 * d] = v.w;
    }
}

template <bool TR>
TFT_DINL u32x4 lds_get_quad(const uint32_t *sm, uint32_t a) {
    if constexpr (TR) {
        return *reinterpret_cast<const u32x4 *>(sm + a);
    } else {
        constexpr uint32_t d = quad_lds_step(false);
        return u32x4{sm[a], sm[a + d], sm[a + 2 * d], sm[a + 3 * d]};
    }
}

template <int C>
TFT_DINL void run_prog(uint32_t *sm, const Job &J, const LeafProg *__restrict__ progs,
                       const LeafStep *__restrict__ steps, const LeafOp *__restrict__ ops, uint32_t ord_mask,
                       uint32_t wave) {
    const Big<C> ar;
    const LeafProg P = progs[J.prog];
    for (uint32_t st = 0; st < P.step_count; ++st) {
        const LeafStep LS = steps[P.step_begin + st];
        for (uint32_t j = wave; j < LS.op_count; j += kThreads / 64u) base_case<C>(ar, sm, ops[LS.op_begin + j], J.s, ord_mask);
        __syncthreads();
    }
}

// One pass: jobs [job_begin, job_begin + njobs), a persistent grid of
// workgroups of 512 threads, each running jobs blockIdx.x, blockIdx.x + gridDim.x, ...
template <int C, bool TR>
__global__ void __launch_bounds__(512) fermat_leaf2_kernel(const Job *__restrict__ jobs,
                                                           const LeafProg *__restrict__ progs,
                                                           const LeafStep *__restrict__ steps,
                                                           const LeafOp *__restrict__ ops, uint32_t *__restrict__ x,
                                                           uint64_t cap, uint32_t ord_mask, uint32_t job_begin,
                                                           uint32_t njobs) {
    constexpr uint32_t W = 64u * C, WQ = W / 4u;
    constexpr int QPT = kQuadsPerThread;
    extern __shared__ uint32_t sm[];
    const uint32_t tid = threadIdx.x;
    const uint32_t wave = uni(tid >> 6);
    uint32_t jb = blockIdx.x;
    if (jb >= njobs) return;
    uint32_t *tops = x + cap * W;

    u32x4 pre[QPT];
    uint32_t pre_top = 0;
    const QuadMap<C, TR> qm(tid);
    Job J = jobs[job_begin + jb];
#pragma unroll
    for (int i = 0; i < QPT; ++i)
        if (qm.valid(J.nload, i)) pre[i] = *reinterpret_cast<const u32x4 *>(x + qm.global(J, i));
    if (tid < J.nload) pre_top = tops[J.base + (uint64_t)tid * J.stride];
#pragma unroll
    for (int i = 0; i < QPT; ++i)
        if (qm.valid(J.nload, i)) lds_put_quad<TR>(sm, qm.lds(i), pre[i]);
    if (tid < J.nload) sm[tid] = pre_top;
    __syncthreads();

    for (;;) {
        const uint32_t jn = jb + gridDim.x;
        const bool has_next = jn < njobs;
        Job JN = J;
        if (has_next) {
            JN = jobs[job_begin + jn];
#pragma unroll
            for (int i = 0; i < QPT; ++i)
                if (qm.valid(JN.nload, i)) pre[i] = *reinterpret_cast<const u32x4 *>(x + qm.global(JN, i));
            if (tid < JN.nload) pre_top = tops[JN.base + (uint64_t)tid * JN.stride];
        }

        run_prog<C>(sm, J, progs, steps, ops, ord_mask, wave);

        // outputs of J leave LDS while the inputs of JN take their place; a
        // thread reads and writes only its own quads, so no barrier between
        const uint32_t nin = has_next ? JN.nload : 0u;
        const uint32_t out_top = tid < J.nstore ? sm[tid] : 0u;
        if (tid < nin) sm[tid] = pre_top;
#pragma unroll
        for (int i0 = 0; i0 < QPT; i0 += 4) {
            u32x4 out[4];
#pragma unroll
            for (int i = i0; i < i0 + 4; ++i)
                if (qm.valid(J.nstore, i)) out[i - i0] = lds_get_quad<TR>(sm, qm.lds(i));
#pragma unroll
            for (int i = i0; i < i0 + 4; ++i)
                if (qm.valid(nin, i)) lds_put_quad<TR>(sm, qm.lds(i), pre[i]);
#pragma unroll
            for (int i = i0; i < i0 + 4; ++i)
                if (qm.valid(J.nstore, i)) *reinterpret_cast<u32x4 *>(x + qm.global(J, i)) = out[i - i0];
        }
        if (tid < J.nstore) tops[J.base + (uint64_t)tid * J.stride] = out_top;
        if (!has_next) break;
        __syncthreads();
        J = JN;
        jb = jn;
    }
}

}  // namespace lf2
}  // namespace tft
