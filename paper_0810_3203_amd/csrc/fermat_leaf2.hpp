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
//     stores the next job's inputs, so copies overlap compute within a CU;
//   * small leaves are packed: a workgroup takes `pack` consecutive jobs of the
//     pass at once, job p in LDS cells [p slot, (p+1) slot), so that a pass of
//     4-cell leaves still gives every wave a base case per step.
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

// The jobs a workgroup holds at once: jobs[first .. first + count), job p in
// LDS cells [p << slot_log2, (p+1) << slot_log2).  PK = false: one job (count
// = 1), its descriptor in scalar registers.  PK = true: lane p of every wave
// keeps job p's cell range in registers, and the copy sweeps read a job's
// range with lane reads instead of holding every job in scalar registers.
template <bool PK>
struct Pack {
    uint32_t first, count;
    Job j;                                                           // PK = false
    uint32_t base_lo, base_hi, stride_lo, stride_hi, nload, nstore, prog, s;  // PK: job `lane` (lane < count)
};

template <bool PK>
TFT_DINL Pack<PK> load_pack(const Job *__restrict__ jobs, uint32_t first, uint32_t count) {
    Pack<PK> pk{first, count, Job{}, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
    if constexpr (!PK) {
        pk.j = jobs[first];
    } else {
        const uint32_t l = lane_id();
        if (l < count) {
            const Job J = jobs[first + l];
            pk.base_lo = (uint32_t)J.base;
            pk.base_hi = (uint32_t)(J.base >> 32);
            pk.stride_lo = (uint32_t)J.stride;
            pk.stride_hi = (uint32_t)(J.stride >> 32);
            pk.nload = J.nload;
            pk.nstore = J.nstore;
            pk.prog = J.prog;
            pk.s = J.s;
        }
    }
    return pk;
}

// Cell range of pack cell c (wave-uniform): false if c belongs to no job or
// lies at or beyond the job's input (out: output) cells.
struct CellAt {
    uint64_t base, stride;
    uint32_t local;
};
template <bool PK>
TFT_DINL bool pack_cell(const Pack<PK> &pk, uint32_t slot_log2, uint32_t c, bool out, CellAt &at) {
    if constexpr (!PK) {
        if (pk.count == 0u || c >= (out ? pk.j.nstore : pk.j.nload)) return false;
        at.local = c;
        at.base = pk.j.base;
        at.stride = pk.j.stride;
        return true;
    } else {
        const uint32_t p = c >> slot_log2;
        if (p >= pk.count) return false;
        at.local = c & ((1u << slot_log2) - 1u);
        if (at.local >= (uint32_t)readlane(out ? pk.nstore : pk.nload, (int)p)) return false;
        at.base = (uint64_t)readlane(pk.base_lo, (int)p) | (uint64_t)readlane(pk.base_hi, (int)p) << 32;
        at.stride = (uint64_t)readlane(pk.stride_lo, (int)p) | (uint64_t)readlane(pk.stride_hi, (int)p) << 32;
        return true;
    }
}

template <int C, bool TR>
struct QuadMap {
    static constexpr uint32_t W = 64u * C, K = quad_cells_per_sweep(C);
    uint32_t c0;    // first cell of the thread (the same for the whole wave)
    uint32_t loff;  // LDS dword offset of the thread's quad inside its cell
    uint32_t goff;  // dword offset of the thread's quad inside a global cell
    TFT_DINL explicit QuadMap(uint32_t tid)
        : c0(uni(quad_c0(C, tid))), loff(quad_loff(C, TR, tid)), goff(quad_goff(C, TR, tid)) {}
    // dword index (from x) of the thread's quad in the cell at
    TFT_DINL uint64_t global(const CellAt &at) const { return (at.base + (uint64_t)at.local * at.stride) * W + goff; }
    TFT_DINL uint32_t lds(int i) const { return cell_base(W, c0 + (uint32_t)i * K) + loff; }
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

// Runs the programs of every job of the pack, step by step; step st's base
// cases of all the jobs are one list dealt out to the waves.
template <int C, bool PK>
TFT_DINL void run_pack(uint32_t *sm, const Job *__restrict__ jobs, const Pack<PK> &pk, uint32_t slot_log2,
                       const LeafProg *__restrict__ progs, const LeafStep *__restrict__ steps,
                       const LeafOp *__restrict__ ops, uint32_t ord_mask, uint32_t wave) {
    constexpr uint32_t NW = kThreads / 64u;
    const Big<C> ar;
    if constexpr (!PK) {
        const LeafProg P = progs[pk.j.prog];
        for (uint32_t st = 0; st < P.step_count; ++st) {
            const LeafStep LS = steps[P.step_begin + st];
            for (uint32_t j = wave; j < LS.op_count; j += NW) base_case<C>(ar, sm, ops[LS.op_begin + j], pk.j.s, ord_mask);
            __syncthreads();
        }
        return;
    }
    // jobs of one program (the common case): one program, each step's items
    // are (job, op) pairs dealt out in order
    const uint32_t prog0 = uni(pk.prog);
    if (ballot(lane_id() < pk.count && pk.prog != prog0) == 0ull) {
        const LeafProg P = progs[prog0];
        for (uint32_t st = 0; st < P.step_count; ++st) {
            const LeafStep LS = steps[P.step_begin + st];
            const uint32_t n = LS.op_count;
            uint32_t p = 0, j = wave;
            while (j >= n && p < pk.count) {
                j -= n;
                ++p;
            }
            while (p < pk.count) {
                base_case<C>(ar, sm, ops[LS.op_begin + j], (uint32_t)readlane(pk.s, (int)p), ord_mask, p << slot_log2);
                j += NW;
                while (j >= n && p < pk.count) {
                    j -= n;
                    ++p;
                }
            }
            __syncthreads();
        }
        return;
    }
    uint32_t nsteps = 0;
    for (uint32_t p = 0; p < pk.count; ++p) {
        const uint32_t sc = progs[jobs[pk.first + p].prog].step_count;
        nsteps = sc > nsteps ? sc : nsteps;
    }
    for (uint32_t st = 0; st < nsteps; ++st) {
        uint32_t off = 0;  // items of this step dealt so far
        for (uint32_t p = 0; p < pk.count; ++p) {
            const Job J = jobs[pk.first + p];
            const LeafProg P = progs[J.prog];
            if (st >= P.step_count) continue;
            const LeafStep LS = steps[P.step_begin + st];
            const uint32_t cofs = p << slot_log2;
            for (uint32_t j = (wave + NW - off % NW) % NW; j < LS.op_count; j += NW)
                base_case<C>(ar, sm, ops[LS.op_begin + j], J.s, ord_mask, cofs);
            off += LS.op_count;
        }
        __syncthreads();
    }
}

// One pass: jobs [job_begin, job_begin + njobs) in packs of `pack` consecutive
// jobs (each in 2^slot_log2 LDS cells), a persistent grid of workgroups of 512
// threads, each running packs blockIdx.x, blockIdx.x + gridDim.x, ...
template <int C, bool TR, bool PK>
__global__ void __launch_bounds__(512) fermat_leaf2_kernel(const Job *__restrict__ jobs,
                                                           const LeafProg *__restrict__ progs,
                                                           const LeafStep *__restrict__ steps,
                                                           const LeafOp *__restrict__ ops, uint32_t *__restrict__ x,
                                                           uint64_t cap, uint32_t ord_mask, uint32_t job_begin,
                                                           uint32_t njobs, uint32_t pack, uint32_t slot_log2) {
    constexpr uint32_t W = 64u * C;
    constexpr int QPT = kQuadsPerThread;
    extern __shared__ uint32_t sm[];
    const uint32_t tid = threadIdx.x;
    const uint32_t wave = uni(tid >> 6);
    const uint32_t npacks = (njobs + pack - 1u) / pack;
    uint32_t kb = blockIdx.x;
    if (kb >= npacks) return;
    jobs += job_begin;
    uint32_t *tops = x + cap * W;
    auto pack_at = [&](uint32_t k) {
        const uint32_t first = k * pack;
        return load_pack<PK>(jobs, first, njobs - first < pack ? njobs - first : pack);
    };
    // top word of pack cell tid: its global index, or ~0 if the cell is not an
    // input (out: not an output) of its job
    auto top_index = [&](const Pack<PK> &pk, bool out) -> uint64_t {
        if constexpr (!PK) {
            if (pk.count == 0u) return ~0ull;
            return tid < (out ? pk.j.nstore : pk.j.nload) ? pk.j.base + (uint64_t)tid * pk.j.stride : ~0ull;
        } else {
            const uint32_t p = tid >> slot_log2, local = tid & ((1u << slot_log2) - 1u);
            if (p >= pk.count) return ~0ull;
            const Job J = jobs[pk.first + p];
            return local < (out ? J.nstore : J.nload) ? J.base + (uint64_t)local * J.stride : ~0ull;
        }
    };
    const QuadMap<C, TR> qm(tid);
    auto cell = [&](int i) { return qm.c0 + (uint32_t)i * QuadMap<C, TR>::K; };

    u32x4 pre[QPT];
    uint32_t pre_top = 0;
    Pack<PK> pk = pack_at(kb);
    {
#pragma unroll
        for (int i = 0; i < QPT; ++i) {
            CellAt at;
            if (pack_cell(pk, slot_log2, cell(i), false, at))
                pre[i] = *reinterpret_cast<const u32x4 *>(x + qm.global(at));
        }
        const uint64_t ti = top_index(pk, false);
        if (ti != ~0ull) pre_top = tops[ti];
#pragma unroll
        for (int i = 0; i < QPT; ++i) {
            CellAt at;
            if (pack_cell(pk, slot_log2, cell(i), false, at)) lds_put_quad<TR>(sm, qm.lds(i), pre[i]);
        }
        if (ti != ~0ull) sm[tid] = pre_top;
    }
    __syncthreads();

    for (;;) {
        const uint32_t kn = kb + gridDim.x;
        const bool has_next = kn < npacks;
        Pack<PK> pn{0u, 0u, Job{}, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
        uint64_t tin = ~0ull;
        // The next pack's loads are issued unconditionally: a quad that is no
        // input of it (or every quad after the last pack) reads the thread's
        // quad of cell 0 instead, and its value is never used.  A load under a
        // branch would leave the register a merge of the loaded and the old
        // value, and the compiler resolves that merge with a copy that waits
        // for the load, so the loads would complete before the butterflies
        // start instead of during them.
        if (has_next) pn = pack_at(kn);
        tin = top_index(pn, false);
        pre_top = tops[tin != ~0ull ? tin : 0ull];
#pragma unroll
        for (int i = 0; i < QPT; ++i) {
            CellAt at;
            const uint64_t a = pack_cell(pn, slot_log2, cell(i), false, at) ? qm.global(at) : (uint64_t)qm.goff;
            pre[i] = *reinterpret_cast<const u32x4 *>(x + a);
        }

        run_pack<C, PK>(sm, jobs, pk, slot_log2, progs, steps, ops, ord_mask, wave);

        // outputs of this pack leave LDS while the inputs of the next take their
        // place; a thread reads and writes only its own quads, so no barrier
        // between.  First every quad is swapped (LDS output into the register
        // the input leaves), then all global stores follow: the LDS writes
        // wait for the prefetched loads only, never for a store of the same
        // sweep (both count in vmcnt).
        const uint64_t tout = top_index(pk, true);
        const uint32_t out_top = tout != ~0ull ? sm[tid] : 0u;
        if (tin != ~0ull) sm[tid] = pre_top;
#pragma unroll
        for (int i = 0; i < QPT; ++i) {
            CellAt at;
            u32x4 o = pre[i];
            if (pack_cell(pk, slot_log2, cell(i), true, at)) o = lds_get_quad<TR>(sm, qm.lds(i));
            if (pack_cell(pn, slot_log2, cell(i), false, at)) lds_put_quad<TR>(sm, qm.lds(i), pre[i]);
            pre[i] = o;
        }
#pragma unroll
        for (int i = 0; i < QPT; ++i) {
            CellAt at;
            if (pack_cell(pk, slot_log2, cell(i), true, at)) *reinterpret_cast<u32x4 *>(x + qm.global(at)) = pre[i];
        }
        if (tout != ~0ull) tops[tout] = out_top;
        if (!has_next) break;
        __syncthreads();
        pk = pn;
        kb = kn;
    }
}

}  // namespace lf2
}  // namespace tft
