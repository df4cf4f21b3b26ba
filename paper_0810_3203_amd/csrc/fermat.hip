// HIP kernels for R = Z/(2^N+1) on gfx950: the leaf executor of the
// cache-friendly TFT/ITFT (Alg. 1, Alg. 2), the pointwise products of Sect. 2,
// and the packing of Z[x] coefficients into R (Sect. 5.1).
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
// LDS (cells ESZ dwords apart, limb k at F::addr(k)).  Each thread keeps
// CB 16-byte global accesses in flight before touching LDS.
constexpr int CB = 8;

template <class F, bool IN>
__device__ __forceinline__ void copy_cells(uint32_t *sm, uint32_t *x, const Job &J, uint32_t n, uint32_t tid,
                                           uint32_t nthr) {
    constexpr int W = F::W;
    if constexpr (W % 4 == 0) {
        constexpr uint32_t WQ = W / 4;
        const uint32_t total = n * WQ;
        for (uint32_t q0 = tid; q0 < total; q0 += nthr * CB) {
            uint4 v[CB];
            if (IN) {
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    const uint32_t q = q0 + b * nthr;
                    if (q < total) {
                        const uint32_t cell = q / WQ, off = q % WQ;
                        v[b] = reinterpret_cast<const uint4 *>(x + (J.base + (uint64_t)cell * J.stride) * W)[off];
                    }
                }
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    const uint32_t q = q0 + b * nthr;
                    if (q < total) {
                        const uint32_t cell = q / WQ, k = (q % WQ) * 4u;
                        uint32_t *s = sm + cell * F::ESZ;
                        s[F::addr(k)] = v[b].x;
                        s[F::addr(k + 1)] = v[b].y;
                        s[F::addr(k + 2)] = v[b].z;
                        s[F::addr(k + 3)] = v[b].w;
                    }
                }
            } else {
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    const uint32_t q = q0 + b * nthr;
                    if (q < total) {
                        const uint32_t cell = q / WQ, k = (q % WQ) * 4u;
                        const uint32_t *s = sm + cell * F::ESZ;
                        v[b].x = s[F::addr(k)];
                        v[b].y = s[F::addr(k + 1)];
                        v[b].z = s[F::addr(k + 2)];
                        v[b].w = s[F::addr(k + 3)];
                    }
                }
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    const uint32_t q = q0 + b * nthr;
                    if (q < total) {
                        const uint32_t cell = q / WQ, off = q % WQ;
                        reinterpret_cast<uint4 *>(x + (J.base + (uint64_t)cell * J.stride) * W)[off] = v[b];
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
                sm[cell * F::ESZ + F::addr(off)] = *g;
            else
                *g = sm[cell * F::ESZ + F::addr(off)];
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

template <int S, int C, int V>
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

    copy_cells<F, true>(sm, x, J, J.nload, tid, nthr);
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
                    (uint32_t)((((uint64_t)J.s << (o.w1 >> 24)) + (uint64_t)(o.w1 & 0xFFFFFFu)) & ord_mask);
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

    copy_cells<F, false>(sm, x, J, J.nstore, tid, nthr);
    for (uint32_t t = tid; t < J.nstore; t += nthr) x[cap * W + J.base + (uint64_t)t * J.stride] = stop[t];
}

template <int S, int C, int V>
__global__ void __launch_bounds__(512) fermat_leaf_kernel(const Job *__restrict__ jobs,
                                                           const LeafProg *__restrict__ progs,
                                                           const LeafStep *__restrict__ steps,
                                                           const LeafOp *__restrict__ ops, uint32_t *__restrict__ x,
                                                           uint64_t cap, uint32_t ord_mask, uint32_t lds_cells,
                                                           uint32_t job_offset) {
    leaf_body<S, C, V>(jobs, progs, steps, ops, x, cap, ord_mask, lds_cells, job_offset);
}

// ---------------------------------------------------------------------------
// pointwise products  c = a b 2^scale_e  in Z/(2^N+1)
//
// One workgroup per product.  The negacyclic limb convolution
//   d_k = sum_{i+j=k} a_i b_j - sum_{i+j=k+W} a_i b_j     (2^N = -1)
// is accumulated per output column in 96-bit sums (P_k, N_k), each thread
// owning 8 consecutive columns and sliding a register window over b.  The
// column sums are then folded into four limb vectors PL + HP - NL - HN that
// one wave adds with the carry-lookahead chains, followed by canonicalisation
// and the multiplication by 2^scale_e.
// ---------------------------------------------------------------------------

constexpr int PW_COLS = 8;

// threads of a pointwise workgroup for W limbs: one per PW_COLS columns, 64..256
constexpr uint32_t pw_threads(int W) {
    uint32_t t = (uint32_t)W / PW_COLS;
    t = t < 64 ? 64 : (t > 256 ? 256 : t);
    return (t + 63) / 64 * 64;
}

// c = a b 2^scale_e for one product; a, b, c are W-limb cells (c may alias a or b),
// ta, tb their top words, tc where c's top goes.  Called by a whole workgroup.
template <int S, int C>
__device__ __forceinline__ void pointwise_body(const uint32_t *a, uint32_t ta, const uint32_t *b, uint32_t tb,
                                               uint32_t *c, uint32_t *tc, uint32_t scale_e) {
    using F = FChunk<S, C>;
    constexpr int W = F::W;
    extern __shared__ uint32_t sm[];
    uint32_t *A = sm, *Bv = A + W;
    uint32_t *P0 = Bv + W, *P1 = P0 + W, *P2 = P1 + W, *N0 = P2 + W, *N1 = N0 + W, *N2 = N1 + W;
    uint32_t *Y = N2 + W;  // F::ESZ dwords, LDS layout of one element
    uint32_t &topY = Y[F::ESZ];
    const uint32_t tid = threadIdx.x, nthr = blockDim.x;

    for (uint32_t q = tid; q < (uint32_t)W; q += nthr) {
        A[q] = a[q];
        Bv[q] = b[q];
    }
    __syncthreads();

    const bool special = (ta | tb) != 0u;
    if (!special) {
        // column sums, PW_COLS consecutive columns per thread
        for (uint32_t k0 = tid * PW_COLS; k0 < (uint32_t)W; k0 += nthr * PW_COLS) {
            constexpr int NC = (W < PW_COLS) ? W : PW_COLS;
            uint64_t pl[NC], nl[NC];
            uint32_t ph[NC], nh[NC], bw[NC];
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) {
                pl[cc] = nl[cc] = 0;
                ph[cc] = nh[cc] = 0;
                bw[cc] = Bv[(k0 + cc) & (W - 1)];  // window at i = 0: b_{k0+cc}
            }
            for (uint32_t ii = 0; ii < (uint32_t)W; ++ii) {
                const uint64_t av = A[ii];
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) {
                    const uint64_t pr = av * bw[cc];
                    if (ii <= k0 + cc) {
                        const uint64_t s = pl[cc] + pr;
                        ph[cc] += s < pr ? 1u : 0u;
                        pl[cc] = s;
                    } else {
                        const uint64_t s = nl[cc] + pr;
                        nh[cc] += s < pr ? 1u : 0u;
                        nl[cc] = s;
                    }
                }
                // slide: next i needs b_{k0+cc-(i+1)}
#pragma unroll
                for (int cc = NC - 1; cc > 0; --cc) bw[cc] = bw[cc - 1];
                bw[0] = Bv[(k0 - ii - 1u) & (W - 1)];
            }
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) {
                const uint32_t k = k0 + cc;
                P0[k] = (uint32_t)pl[cc];
                P1[k] = (uint32_t)(pl[cc] >> 32);
                P2[k] = ph[cc];
                N0[k] = (uint32_t)nl[cc];
                N1[k] = (uint32_t)(nl[cc] >> 32);
                N2[k] = nh[cc];
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
    for (uint32_t q = tid; q < (uint32_t)W; q += nthr) c[q] = Y[F::addr(q)];
    if (tid == 0) *tc = topY;
}

template <int S, int C>
__global__ void __launch_bounds__(256) fermat_pointwise_kernel(const uint32_t *__restrict__ a,
                                                               const uint32_t *__restrict__ b, uint32_t *c,
                                                               uint64_t cap, uint32_t scale_e, uint32_t base) {
    constexpr int W = S * C;
    const uint64_t i = (uint64_t)base + blockIdx.x;
    pointwise_body<S, C>(a + i * W, a[cap * W + i], b + i * W, b[cap * W + i], c + i * W, c + cap * W + i, scale_e);
}

// Pointwise products over a list: item i multiplies cells it.x and it.y of the
// cell array x (capacity cap) into cell it.x, with its own scale 2^it.z.
template <int S, int C>
__global__ void __launch_bounds__(256) fermat_pointwise_items_kernel(uint32_t *x, uint64_t cap,
                                                                     const uint4 *__restrict__ items) {
    constexpr int W = S * C;
    const uint4 it = items[blockIdx.x];
    uint32_t *ca = x + (uint64_t)it.x * W, *cb = x + (uint64_t)it.y * W;
    pointwise_body<S, C>(ca, x[cap * W + it.x], cb, x[cap * W + it.y], ca, x + cap * W + it.x, it.z);
}

// Pack: cell e of an operand holds coefficients e*k .. e*k+k-1, coefficient
// e*k+j in limbs [j*ws, j*ws + climbs) (slot j), zeros elsewhere (Sect. 5.1 with
// k = 1; k > 1 bundles k coefficients per ring element).  One descriptor per
// operand, blockIdx.y selects it.
__global__ void fermat_pack_kernel(const PackDesc *__restrict__ descs, PackDesc inl, uint32_t *__restrict__ x,
                                   uint64_t cap, uint32_t W) {
    const PackDesc d = descs ? descs[blockIdx.y] : inl;
    const uint64_t total = d.z * (uint64_t)W;
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < total;
         q += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t e = q / W;
        const uint32_t p = (uint32_t)(q % W);
        const uint32_t j = p / d.ws, off = p % d.ws;
        const uint64_t c = e * d.k + j;
        x[(d.cell0 + e) * W + p] = (j < d.k && off < d.climbs && c < d.len) ? d.coef[c * d.climbs + off] : 0u;
        if (p == 0) x[cap * W + d.cell0 + e] = 0u;
    }
}

// Unpack with k = 1: coefficient t is the low limbs of cell t.
__global__ void fermat_unpack1_kernel(const UnpackDesc *__restrict__ descs, UnpackDesc inl,
                                      const uint32_t *__restrict__ x, uint64_t cap, uint32_t W) {
    const UnpackDesc d = descs ? descs[blockIdx.y] : inl;
    const uint64_t total = d.len_out * (uint64_t)d.olimbs;
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < total;
         q += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t t = q / d.olimbs;
        const uint32_t i = (uint32_t)(q % d.olimbs);
        const uint64_t cell = d.cell0 + t;
        d.out[q] = i < W ? x[cell * W + i] : (i == W ? x[cap * W + cell] : 0u);
    }
}

// Unpack with k > 1: the product cell m holds slots 0..2k-2 of width ws limbs;
// coefficient t = m k + j is slot j of cell m plus slot j + k of cell m - 1.
__global__ void fermat_unpackk_kernel(const UnpackDesc *__restrict__ descs, UnpackDesc inl,
                                      const uint32_t *__restrict__ x, uint32_t W) {
    const UnpackDesc d = descs ? descs[blockIdx.y] : inl;
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < d.len_out;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t m = t / d.k;
        const uint32_t j = (uint32_t)(t % d.k);
        const uint32_t *s0 = (m < d.ncells) ? x + (d.cell0 + m) * W + (uint64_t)j * d.ws : nullptr;
        const uint32_t *s1 = (m >= 1 && j + 1 < d.k && m - 1 < d.ncells)
                                 ? x + (d.cell0 + m - 1) * W + (uint64_t)(j + d.k) * d.ws
                                 : nullptr;
        uint32_t *o = d.out + t * d.olimbs;
        uint64_t c = 0;
        for (uint32_t i = 0; i < d.olimbs; ++i) {
            if (i < d.ws) {
                c += (s0 ? s0[i] : 0u);
                c += (s1 ? s1[i] : 0u);
            }
            o[i] = (uint32_t)c;
            c >>= 32;
        }
    }
}

template <int S, int C, int V>
hipError_t leaf_launch_set(uint32_t nwaves, uint32_t njobs, uint32_t lds_cells, const Job *jobs, uint32_t job_offset,
                           const LeafProg *progs, const LeafStep *steps, const LeafOp *ops, uint32_t *x, uint64_t cap,
                           uint32_t ord_mask, hipStream_t st) {
    const size_t lds = (size_t)lds_cells * (FChunk<S, C>::ESZ + 1) * 4;
    if (lds > kLdsBudget - kLeafStaticLds) return hipErrorInvalidValue;
    auto kern = &fermat_leaf_kernel<S, C, V>;
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

template <int S, int C>
hipError_t leaf_launch(uint32_t nwaves, uint32_t njobs, uint32_t lds_cells, const Job *jobs, uint32_t job_offset,
                       const LeafProg *progs, const LeafStep *steps, const LeafOp *ops, uint32_t *x, uint64_t cap,
                       uint32_t ord_mask, uint32_t opmask, hipStream_t st) {
    if ((opmask & ~kTftOps) == 0u)
        return leaf_launch_set<S, C, SET_TFT>(nwaves, njobs, lds_cells, jobs, job_offset, progs, steps, ops, x, cap,
                                              ord_mask, st);
    if ((opmask & ~kItftOps) == 0u)
        return leaf_launch_set<S, C, SET_ITFT>(nwaves, njobs, lds_cells, jobs, job_offset, progs, steps, ops, x, cap,
                                               ord_mask, st);
    return leaf_launch_set<S, C, SET_ALL>(nwaves, njobs, lds_cells, jobs, job_offset, progs, steps, ops, x, cap,
                                          ord_mask, st);
}

template <class KernelT>
hipError_t pointwise_attr(KernelT *kern, size_t lds, bool &done) {
    if (done || lds <= 65536) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
    if (e == hipSuccess) done = true;
    return e;
}

template <int S, int C>
hipError_t pointwise_launch(uint64_t n, const uint32_t *a, const uint32_t *b, uint32_t *c, uint64_t cap,
                            uint32_t scale_e, hipStream_t st) {
    constexpr int W = S * C;
    const size_t lds = (size_t)(8 * W + FChunk<S, C>::ESZ + 1) * 4;
    if (lds > kLdsBudget) return hipErrorInvalidValue;
    static bool attr = false;
    hipError_t e = pointwise_attr(&fermat_pointwise_kernel<S, C>, lds, attr);
    if (e != hipSuccess) return e;
    const uint64_t per = kMaxGridX / pw_threads(W);
    for (uint64_t i0 = 0; i0 < n; i0 += per) {
        const uint64_t nb = n - i0 < per ? n - i0 : per;
        hipLaunchKernelGGL((fermat_pointwise_kernel<S, C>), dim3((uint32_t)nb), dim3(pw_threads(W)), lds, st, a, b,
                           c, cap, scale_e, (uint32_t)i0);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int S, int C>
hipError_t pointwise_items_launch(uint64_t nitems, uint32_t *x, uint64_t cap, const uint4 *items, hipStream_t st) {
    constexpr int W = S * C;
    const size_t lds = (size_t)(8 * W + FChunk<S, C>::ESZ + 1) * 4;
    if (lds > kLdsBudget) return hipErrorInvalidValue;
    static bool attr = false;
    hipError_t e = pointwise_attr(&fermat_pointwise_items_kernel<S, C>, lds, attr);
    if (e != hipSuccess) return e;
    const uint64_t per = kMaxGridX / pw_threads(W);
    for (uint64_t i0 = 0; i0 < nitems; i0 += per) {
        const uint64_t nb = nitems - i0 < per ? nitems - i0 : per;
        hipLaunchKernelGGL((fermat_pointwise_items_kernel<S, C>), dim3((uint32_t)nb), dim3(pw_threads(W)), lds, st,
                           x, cap, items + i0);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

uint32_t lds_budget_bytes() { return kLdsBudget - kLeafStaticLds; }

uint32_t fermat_lds_cell_bytes(uint32_t W) {
    const uint32_t S = W < 64 ? W : 64, C = W / S;
    const uint32_t CP = C > 1 ? C + 1 : 1;
    return 4u * (S * CP + 1u);
}

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

hipError_t launch_fermat_leaf(uint32_t W, uint32_t nwaves, uint32_t njobs, uint32_t lds_cells, const Job *jobs,
                              uint32_t job_offset, const LeafProg *progs, const LeafStep *steps, const LeafOp *ops,
                              uint32_t *x, uint64_t cap, uint32_t ord_mask, uint32_t opmask, hipStream_t st) {
    if (njobs == 0) return hipSuccess;
    TFT_FERMAT_DISPATCH(W, leaf_launch, nwaves, njobs, lds_cells, jobs, job_offset, progs, steps, ops, x, cap,
                        ord_mask, opmask, st)
}

hipError_t launch_fermat_pointwise(uint32_t W, uint64_t n, const uint32_t *a, const uint32_t *b, uint32_t *c,
                                   uint64_t cap, uint32_t scale_e, hipStream_t st) {
    if (n == 0) return hipSuccess;
    TFT_FERMAT_DISPATCH(W, pointwise_launch, n, a, b, c, cap, scale_e, st)
}

hipError_t launch_fermat_pointwise_items(uint32_t W, uint64_t nitems, uint32_t *x, uint64_t cap, const uint4 *items,
                                         hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    TFT_FERMAT_DISPATCH(W, pointwise_items_launch, nitems, x, cap, items, st)
}

hipError_t launch_fermat_pack(uint32_t W, const PackDesc *descs, uint32_t ndesc, const PackDesc &inl, uint64_t max_z,
                              uint32_t *x, uint64_t cap, hipStream_t st) {
    if (ndesc == 0 || max_z == 0) return hipSuccess;
    uint64_t blocks = (max_z * W + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fermat_pack_kernel, dim3((uint32_t)blocks, ndesc), dim3(256), 0, st, descs, inl, x, cap, W);
    return hipGetLastError();
}

hipError_t launch_fermat_unpack(uint32_t W, const UnpackDesc *descs, uint32_t ndesc, const UnpackDesc &inl,
                                uint64_t max_len, uint32_t max_olimbs, bool bundled, const uint32_t *x, uint64_t cap,
                                hipStream_t st) {
    if (ndesc == 0 || max_len == 0) return hipSuccess;
    if (!bundled) {
        uint64_t blocks = (max_len * max_olimbs + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(fermat_unpack1_kernel, dim3((uint32_t)blocks, ndesc), dim3(256), 0, st, descs, inl, x, cap,
                           W);
    } else {
        uint64_t blocks = (max_len + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(fermat_unpackk_kernel, dim3((uint32_t)blocks, ndesc), dim3(256), 0, st, descs, inl, x, W);
    }
    return hipGetLastError();
}

}  // namespace tft
