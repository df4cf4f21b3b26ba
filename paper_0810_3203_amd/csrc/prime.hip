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

constexpr uint32_t kZpThreads = 512;
constexpr uint32_t kZpLdsWords = 40896;  // 160 KB, one compute unit's LDS, less the static words of __syncthreads_or
constexpr uint32_t kZpPairWords = 20416;  // two workgroups on a compute unit
constexpr uint32_t kZpCUs = 256;        // compute units of the part (MI355X)
constexpr uint32_t kDescWords = 8;       // base lo, base hi, stride lo, stride hi, nload, nstore, prog, s

// theta^e in Montgomery form for 0 <= e < 2^27 from three tables of 512
// entries: e = e0 + 2^9 e1 + 2^18 e2 and v[k][j] = theta^(j 2^(9k)).  Built
// by repeated multiplication at compile time.
struct ThetaPowTab {
    uint32_t v[3][512];
};
constexpr ThetaPowTab make_theta_pow_tab() {
    ThetaPowTab t{};
    for (int k = 0; k < 3; ++k) {
        const uint32_t g = zp::theta_pow_m(1ull << (9 * k));
        uint32_t x = zp::to_mont(1u);
        for (int j = 0; j < 512; ++j) {
            t.v[k][j] = x;
            x = zp::mont(x, g);
        }
    }
    return t;
}
__constant__ ThetaPowTab kThetaPow = make_theta_pow_tab();

__device__ __forceinline__ uint32_t theta_pow_tab(uint32_t e) {
    return zp::mont(zp::mont(kThetaPow.v[0][e & 511u], kThetaPow.v[1][(e >> 9) & 511u]), kThetaPow.v[2][e >> 18]);
}

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

// Where the jobs of a pack keep their cells and twist tables in LDS.
struct PackLds {
    uint32_t *dat;       // job p's cells at p * pitch
    uint32_t pitch;
    const uint32_t *zt;  // job p's table at p * 2 zw: theta^(s 2^a), then theta^(-s 2^a)
    uint32_t zw;
    bool uni;            // every job of the pack has the same twist s (a row pass)
};

// One base case (cells i0, i1; twiddle theta^(s 2^alog) times tw, tw = theta^b
// or theta^-b) on jobs p0 .. p1-1 of a pack.  With one twist for the whole
// pack (UNI) the twiddle is formed once.
template <uint32_t CODE, bool UNI>
__device__ __forceinline__ void zp_jobs(const PackLds &L, uint32_t p0, uint32_t p1, uint32_t i0, uint32_t i1,
                                        uint32_t alog, uint32_t tw) {
    constexpr bool TW = CODE == OP_T22 || CODE == OP_T21 || CODE == OP_I2 || CODE == OP_I1F1Z2 || CODE == OP_I1F1Z1;
    const uint32_t zoff = (CODE == OP_I2 ? L.zw : 0u) + alog;
    const uint32_t z0 = TW && UNI ? zp::mont(L.zt[zoff], tw) : 0u;
    for (uint32_t p = p0; p < p1; ++p) {
        const uint32_t zm = !TW ? 0u : UNI ? z0 : zp::mont(L.zt[2u * L.zw * p + zoff], tw);
        zp_base_case(L.dat + p * L.pitch, CODE, i0, i1, zm);
    }
}

template <bool UNI>
__device__ __forceinline__ void zp_jobs_code(uint32_t code, const PackLds &L, uint32_t p0, uint32_t p1, uint32_t i0,
                                             uint32_t i1, uint32_t alog, uint32_t tw) {
    switch (code) {
        case OP_T22: zp_jobs<OP_T22, UNI>(L, p0, p1, i0, i1, alog, tw); break;
        case OP_T21: zp_jobs<OP_T21, UNI>(L, p0, p1, i0, i1, alog, tw); break;
        case OP_T12: zp_jobs<OP_T12, UNI>(L, p0, p1, i0, i1, alog, tw); break;
        case OP_I2: zp_jobs<OP_I2, UNI>(L, p0, p1, i0, i1, alog, tw); break;
        case OP_I1F1Z2: zp_jobs<OP_I1F1Z2, UNI>(L, p0, p1, i0, i1, alog, tw); break;
        case OP_I1F1Z1: zp_jobs<OP_I1F1Z1, UNI>(L, p0, p1, i0, i1, alog, tw); break;
        case OP_I1F0Z2: zp_jobs<OP_I1F0Z2, UNI>(L, p0, p1, i0, i1, alog, tw); break;
        case OP_I1F0Z1: zp_jobs<OP_I1F0Z1, UNI>(L, p0, p1, i0, i1, alog, tw); break;
        case OP_I0Z2: zp_jobs<OP_I0Z2, UNI>(L, p0, p1, i0, i1, alog, tw); break;
        case OP_I0Z1: zp_jobs<OP_I0Z1, UNI>(L, p0, p1, i0, i1, alog, tw); break;
        default: break;
    }
}

// Op o of a step on jobs p0 .. p1-1.  A step's ops are grouped by opcode, so a
// wave's lanes mostly share it: then the opcode is taken as a wave-uniform
// value and the dispatch costs scalar branches only.
template <bool UNI>
__device__ __forceinline__ void zp_op_t(const LeafOp &o, uint32_t tw, const PackLds &L, uint32_t p0, uint32_t p1) {
    const uint32_t code = o.w0 & 15u;
    const uint32_t i0 = (o.w0 >> 4) & 16383u, i1 = (o.w0 >> 18) & 16383u;
    const uint32_t alog = op_alog(o);
    const uint32_t c0 = __builtin_amdgcn_readfirstlane(code);
    if (__builtin_amdgcn_ballot_w64(code != c0) == 0)
        zp_jobs_code<UNI>(c0, L, p0, p1, i0, i1, alog, tw);
    else
        zp_jobs_code<UNI>(code, L, p0, p1, i0, i1, alog, tw);
}

__device__ __forceinline__ void zp_op(const LeafOp &o, uint32_t tw, const PackLds &L, uint32_t p0, uint32_t p1) {
    if (L.uni)
        zp_op_t<true>(o, tw, L, p0, p1);
    else
        zp_op_t<false>(o, tw, L, p0, p1);
}

// floor(k / d) for k < 2^24 and 1 <= d < 2^24 (a float estimate, then one correction)
__device__ __forceinline__ uint32_t div_small(uint32_t k, uint32_t d, float rd) {
    uint32_t q = (uint32_t)((float)k * rd);
    if (q * d > k) --q;
    else if ((q + 1u) * d <= k) ++q;
    return q;
}

// A workgroup runs a pack of jobs [first, first + count) of a pass, at most
// 2^pack_log2 jobs of at most 2^slot_log2 cells; zw = twist entries per job
// (every op's alog < zw).  stage_cap > 0 (at least the widest step of the
// pass) gives LDS room for that many ops, three words each: a pass of few
// workgroups, one a compute unit, then copies its program's ops into LDS a
// chunk of whole steps at a time instead of waiting on global memory at every
// step.  Workgroups are numbered so that each XCD (the
// hardware deals workgroup b to XCD b mod 8) takes a contiguous range of
// packs: adjacent columns then share that XCD's L2.
__global__ void __launch_bounds__(kZpThreads) zp_leaf_kernel(const Job *__restrict__ jobs,
                                                             const LeafProg *__restrict__ progs,
                                                             const LeafStep *__restrict__ steps,
                                                             const LeafOp *__restrict__ ops,
                                                             const uint32_t *__restrict__ optw,
                                                             uint32_t *__restrict__ x, uint32_t job_begin,
                                                             uint32_t njobs, uint32_t pack_log2, uint32_t slot_log2,
                                                             uint32_t zw, uint32_t stage_cap) {
    extern __shared__ uint32_t sm[];
    const uint32_t tid = threadIdx.x;
    const uint32_t G = gridDim.x, b = blockIdx.x, xcd = b & 7u, per = G >> 3, rem = G & 7u;
    const uint32_t wg = (xcd < rem ? xcd * (per + 1u) : rem * (per + 1u) + (xcd - rem) * per) + (b >> 3);
    const uint32_t pack = 1u << pack_log2, slot = 1u << slot_log2, pitch = slot + 1u;
    const uint32_t first = wg << pack_log2;
    const uint32_t count = njobs - first < pack ? njobs - first : pack;
    jobs += job_begin + first;
    uint32_t *dsc = sm;                          // kDescWords per job
    uint32_t *ztab = dsc + kDescWords * pack;    // 2 zw per job
    uint32_t *dat = ztab + 2u * zw * pack;
    uint32_t *stage = dat + pack * pitch;        // stage_cap ops: w0, w1, twiddle

    const uint32_t prog0 = jobs[0].prog, s0 = jobs[0].s;
    int mixed = 0, twists = 0;
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
        mixed |= J.prog != prog0;
        twists |= J.s != s0;
    }
    const uint32_t zs = 2u * zw;
    const float rzs = 1.0f / (float)zs;
    for (uint32_t q = tid; q < count * zs; q += kZpThreads) {
        const uint32_t p = div_small(q, zs, rzs), a = q - p * zs;
        const uint32_t e = (jobs[p].s << (a < zw ? a : a - zw)) & (zp::ORD - 1u);
        ztab[q] = theta_pow_tab(a < zw ? e : (zp::ORD - e) & (zp::ORD - 1u));
    }
    mixed = __syncthreads_or(mixed);
    const PackLds L{dat, pitch, ztab, zw, __syncthreads_or(twists) == 0};

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
    // eight loads in flight per thread before their LDS stores.  Loads and
    // stores are unconditional: an element that is no input reads cell 0 of
    // job 0 and stores into job 0's pad word (LDS word `slot`, never read),
    // so that the compiler cannot sink each load into a branch of its own
    // store, where every load would wait for the one before.
    for (uint32_t e0 = tid; e0 < E; e0 += 8u * kZpThreads) {
        uint32_t v[8], at[8];
#pragma unroll
        for (uint32_t u = 0; u < 8u; ++u) {
            const uint32_t e = e0 + u * kZpThreads;
            uint32_t p = 0, r = 0;
            if (e < E) elem(e, p, r);
            const bool in = e < E && p < count && r < dsc[kDescWords * p + 4];
            at[u] = in ? p * pitch + r : slot;
            v[u] = x[in ? gaddr(p, r) : gaddr(0u, 0u)];
        }
#pragma unroll
        for (uint32_t u = 0; u < 8u; ++u) dat[at[u]] = v[u];
    }
    __syncthreads();

    const LeafProg P = progs[prog0];
    if (!mixed && P.step_count && stage_cap) {
        // ops staged in LDS: when a step's ops run past the staged window,
        // the window moves to start at that step and takes as many ops as fit
        const LeafStep SL = steps[P.step_begin + P.step_count - 1u];
        const uint32_t op_end = SL.op_begin + SL.op_count;
        uint32_t cb = 0, ce = 0;
        for (uint32_t st = 0; st < P.step_count; ++st) {
            const LeafStep LS = steps[P.step_begin + st];
            const uint32_t ob = LS.op_begin, oc = LS.op_count;
            if (ob + oc > ce) {
                cb = ob;
                ce = op_end - cb < stage_cap ? op_end : cb + stage_cap;
                for (uint32_t j0 = tid; j0 < ce - cb; j0 += 4u * kZpThreads) {
                    LeafOp o[4];
                    uint32_t t[4];
#pragma unroll
                    for (uint32_t u = 0; u < 4u; ++u) {
                        const uint32_t j = j0 + u * kZpThreads;
                        if (j < ce - cb) {
                            o[u] = ops[cb + j];
                            t[u] = optw[cb + j];
                        }
                    }
#pragma unroll
                    for (uint32_t u = 0; u < 4u; ++u) {
                        const uint32_t j = j0 + u * kZpThreads;
                        if (j < ce - cb) {
                            stage[3u * j] = o[u].w0;
                            stage[3u * j + 1u] = o[u].w1;
                            stage[3u * j + 2u] = t[u];
                        }
                    }
                }
                __syncthreads();
            }
            const uint32_t *sg = stage + 3u * (ob - cb);
            if (count == 1u || 2u * oc >= kZpThreads) {
                for (uint32_t j = tid; j < oc; j += kZpThreads)
                    zp_op(LeafOp{sg[3u * j], sg[3u * j + 1u]}, sg[3u * j + 2u], L, 0u, count);
            } else {
                const float rd = 1.0f / (float)oc;
                for (uint32_t k = tid; k < count * oc; k += kZpThreads) {
                    const uint32_t p = div_small(k, oc, rd), j = k - p * oc;
                    zp_op(LeafOp{sg[3u * j], sg[3u * j + 1u]}, sg[3u * j + 2u], L, p, p + 1u);
                }
            }
            __syncthreads();
        }
    } else if (!mixed && P.step_count) {
        // one program for the whole pack (a program of no steps, a transform
        // whose base cases are all no-ops, leaves the cells as loaded).  Wide steps: a thread takes an op and
        // runs it on every job of the pack (the op is read once); narrow
        // steps: items (job, op) with the op varying fastest.  A program's
        // steps keep their ops back to back, so the next step's ops (up to
        // kPre a thread) are loaded while this step runs, bounded by the
        // program's last op.
        constexpr uint32_t kPre = 4;
        const LeafStep S0 = steps[P.step_begin], SL = steps[P.step_begin + P.step_count - 1u];
        const uint32_t op_end = SL.op_begin + SL.op_count;
        LeafOp po[kPre];
        uint32_t pt[kPre];
        auto fetch = [&](uint32_t ob, LeafOp *o, uint32_t *t) {
#pragma unroll
            for (uint32_t i = 0; i < kPre; ++i) {
                const uint32_t j = ob + tid + i * kZpThreads;
                if (j < op_end) {
                    o[i] = ops[j];
                    t[i] = optw[j];
                }
            }
        };
        fetch(S0.op_begin, po, pt);
        uint32_t ob = S0.op_begin, oc = S0.op_count;
        for (uint32_t st = 0; st < P.step_count; ++st) {
            const uint32_t nb = ob + oc;
            const uint32_t noc = st + 1u < P.step_count ? steps[P.step_begin + st + 1u].op_count : 0u;
            LeafOp no[kPre];
            uint32_t nt[kPre];
            fetch(nb, no, nt);
            if (count == 1u || 2u * oc >= kZpThreads) {
#pragma unroll
                for (uint32_t i = 0; i < kPre; ++i)
                    if (tid + i * kZpThreads < oc) zp_op(po[i], pt[i], L, 0u, count);
                for (uint32_t j = tid + kPre * kZpThreads; j < oc; j += kZpThreads)
                    zp_op(ops[ob + j], optw[ob + j], L, 0u, count);
            } else {
                const float rd = 1.0f / (float)oc;
                for (uint32_t k = tid; k < count * oc; k += kZpThreads) {
                    const uint32_t p = div_small(k, oc, rd), j = k - p * oc;
                    zp_op(ops[ob + j], optw[ob + j], L, p, p + 1u);
                }
            }
            __syncthreads();
#pragma unroll
            for (uint32_t i = 0; i < kPre; ++i) {
                po[i] = no[i];
                pt[i] = nt[i];
            }
            ob = nb;
            oc = noc;
        }
    } else if (mixed) {
        for (uint32_t p = 0; p < count; ++p) {
            const LeafProg Q = progs[dsc[kDescWords * p + 6]];
            for (uint32_t st = 0; st < Q.step_count; ++st) {
                const LeafStep LS = steps[Q.step_begin + st];
                for (uint32_t j = tid; j < LS.op_count; j += kZpThreads)
                    zp_op(ops[LS.op_begin + j], optw[LS.op_begin + j], L, p, p + 1u);
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
    // two workgroups on a compute unit when a job fits half its LDS, else one
    const uint32_t budget = per <= kZpPairWords ? kZpPairWords : kZpLdsWords;
    uint32_t pl = 0;
    while ((2u << pl) * per <= budget && (2u << pl) <= 256u) ++pl;
    // about two packs per workgroup slot (256 compute units, two slots each)
    // when the pass has the jobs
    while (pl > 0 && (njobs >> pl) < 1024u) --pl;
    return pl;
}

hipError_t launch_zp_leaf(uint32_t njobs, uint32_t max_len, uint32_t max_ops, const Job *jobs, uint32_t job_begin,
                          const LeafProg *progs, const LeafStep *steps, const LeafOp *ops, const uint32_t *optw,
                          uint32_t *x, uint32_t zw, hipStream_t st) {
    if (njobs == 0) return hipSuccess;
    uint32_t sl = 0;
    while ((1u << sl) < max_len) ++sl;
    if ((1u << sl) != max_len || zw == 0 || zw > 16) return hipErrorInvalidValue;
    const uint32_t pl = zp_leaf_pack_log2(njobs, sl, zw);
    const uint32_t pack = 1u << pl;
    size_t words = (size_t)pack * (kDescWords + 2u * zw + max_len + 1u);
    if (words > kZpLdsWords) return hipErrorInvalidValue;
    const uint32_t grid = (njobs + pack - 1u) >> pl;
    // no more workgroups than compute units: each has a compute unit's LDS,
    // and the rest of it holds staged ops if the widest step fits
    uint32_t stage_cap = 0;
    if (grid <= kZpCUs) {
        const uint32_t cap = (uint32_t)((kZpLdsWords - words) / 3u);
        if (max_ops && cap >= max_ops) stage_cap = cap;
    }
    words += 3u * (size_t)stage_cap;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&zp_leaf_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kZpLdsWords * 4u));
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(zp_leaf_kernel, dim3(grid), dim3(kZpThreads), words * 4u, st, jobs, progs, steps, ops, optw, x,
                       job_begin, njobs, pl, sl, zw, stage_cap);
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
