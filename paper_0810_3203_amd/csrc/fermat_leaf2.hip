// Instantiations and launcher of the persistent leaf executor (fermat_leaf2.hpp)
// for elements of 1024 and 2048 limbs (transforms) and 256 to 2048 limbs (the
// single-base-case probes), both global cell layouts.
#include "fermat_leaf2.hpp"

namespace tft {

namespace {

constexpr uint32_t kLds = 160u * 1024u;

uint32_t device_cus() {
    static int cache[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cache[dev]) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
        cache[dev] = cus;
    }
    return (uint32_t)cache[dev];
}

// Jobs packed per workgroup for a pass of leaves of `slot` cells: as many as
// the cells the kernel can hold (LDS, and 16 quads per thread), but never so
// many that fewer packs than compute units remain.  Leaves of 8 cells and more
// give at least half of the 8 waves a base case per step and are not packed
// (measured: packing pairs of 8-cell leaves is slower than running them alone).
uint32_t leaf2_pack(uint32_t W, uint32_t njobs, uint32_t slot) {
    if (slot >= 8u) return 1u;
    const uint32_t cap_quads = (uint32_t)lf2::kQuadsPerThread * lf2::kThreads / (W / 4u);
    uint32_t cap_lds = 0;
    while (lf2::lds_dwords(W, cap_lds + 1u) * 4u <= kLds) cap_lds++;
    uint32_t cap = cap_quads < cap_lds ? cap_quads : cap_lds;
    cap = cap < W ? cap : W;  // top words of the cells fit the guard block
    uint32_t pack = cap / slot;
    const uint32_t fill = njobs / device_cus();
    if (pack > fill) pack = fill;
    return pack < 1u ? 1u : pack;
}

template <int C, bool TR>
hipError_t leaf2_launch(uint32_t njobs, uint32_t slot, const Job *jobs, uint32_t job_offset, const LeafProg *progs,
                        const LeafStep *steps, const LeafOp *ops, uint32_t *x, uint64_t cap, uint32_t ord_mask,
                        hipStream_t st) {
    constexpr uint32_t W = 64u * C;
    uint32_t slot_log2 = 0;
    while ((1u << slot_log2) < slot) slot_log2++;
    if (slot == 0u || (1u << slot_log2) != slot) return hipErrorInvalidValue;
    const uint32_t pack = leaf2_pack(W, njobs, slot);
    const uint32_t lds_cells = pack * slot;
    if (lds_cells * (W / 4u) > (uint32_t)lf2::kQuadsPerThread * lf2::kThreads || lds_cells > W)
        return hipErrorInvalidValue;
    const size_t lds = (size_t)lf2::lds_dwords(W, lds_cells) * 4u;
    if (lds > kLds) return hipErrorInvalidValue;
    auto kern = pack > 1u ? &lf2::fermat_leaf2_kernel<C, TR, true> : &lf2::fermat_leaf2_kernel<C, TR, false>;
    static bool attr[2] = {false, false};
    if (!attr[pack > 1u]) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLds);
        if (e != hipSuccess) return e;
        attr[pack > 1u] = true;
    }
    const uint32_t npacks = (njobs + pack - 1u) / pack;
    const uint32_t grid = npacks < device_cus() ? npacks : device_cus();
    hipLaunchKernelGGL(kern, dim3(grid), dim3(lf2::kThreads), lds, st, jobs, progs, steps, ops, x, cap, ord_mask,
                       job_offset, njobs, pack, slot_log2);
    return hipGetLastError();
}

// One base case per workgroup of one wave: record c holds the opcode, the
// exponent, the two top words and the two cells (plain limb order).
template <int C>
__global__ void __launch_bounds__(64) base_case_probe_kernel(const uint32_t *__restrict__ in,
                                                              uint32_t *__restrict__ out, uint32_t ncases) {
    constexpr uint32_t W = 64u * C, REC = 4u + 2u * W;
    extern __shared__ uint32_t sm[];
    const uint32_t c = blockIdx.x;
    if (c >= ncases) return;
    const uint32_t *r = in + (size_t)c * REC;
    const uint32_t l = threadIdx.x;
    for (uint32_t k = l; k < W; k += 64u) {
        sm[lf2::cell_base(W, 0) + lf2::limb_pos(C, k)] = r[4 + k];
        sm[lf2::cell_base(W, 1) + lf2::limb_pos(C, k)] = r[4 + W + k];
    }
    if (l < 2u) sm[l] = r[2 + l];
    __syncthreads();
    const lf2::Big<C> ar;
    const LeafOp o{(r[0] & 15u) | (0u << 4) | (1u << 18), 0u};
    lf2::base_case<C>(ar, sm, o, r[1], 64u * W - 1u);
    __syncthreads();
    uint32_t *w = out + (size_t)c * REC;
    for (uint32_t k = l; k < W; k += 64u) {
        w[4 + k] = sm[lf2::cell_base(W, 0) + lf2::limb_pos(C, k)];
        w[4 + W + k] = sm[lf2::cell_base(W, 1) + lf2::limb_pos(C, k)];
    }
    if (l < 2u) {
        w[2 + l] = sm[l];
        w[l] = r[l];
    }
}

template <int C>
hipError_t probe_launch(uint32_t ncases, const uint32_t *in, uint32_t *out, hipStream_t st) {
    constexpr uint32_t W = 64u * C;
    hipLaunchKernelGGL(base_case_probe_kernel<C>, dim3(ncases), dim3(64), lf2::lds_dwords(W, 2) * 4u, st, in, out,
                       ncases);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_base_case_probe(uint32_t W, uint32_t ncases, const uint32_t *in, uint32_t *out, hipStream_t st) {
    if (ncases == 0) return hipSuccess;
    switch (W) {
        case 256: return probe_launch<4>(ncases, in, out, st);
        case 512: return probe_launch<8>(ncases, in, out, st);
        case 1024: return probe_launch<16>(ncases, in, out, st);
        case 2048: return probe_launch<32>(ncases, in, out, st);
        default: return hipErrorInvalidValue;
    }
}

// The persistent executor pays off for cells of 4 KB and more; for 256 and
// 512 limbs the first leaf kernel runs the short, mixed passes of batched
// products faster (measured on the 4096-request batch: 760 ms against 1273 ms
// with this executor), so transforms of those sizes stay there.
bool fermat_leaf2_supported(uint32_t W) { return W == 1024u || W == 2048u; }

hipError_t launch_fermat_leaf2(uint32_t W, uint32_t njobs, uint32_t lds_cells, const Job *jobs, uint32_t job_offset,
                               const LeafProg *progs, const LeafStep *steps, const LeafOp *ops, uint32_t *x,
                               uint64_t cap, uint32_t ord_mask, uint32_t opmask, bool transposed, hipStream_t st) {
    (void)opmask;  // one kernel runs every base case
    if (njobs == 0) return hipSuccess;
#define TFT_LEAF2_CASE(CC)                                                                                        \
    case 64 * CC:                                                                                                 \
        return transposed ? leaf2_launch<CC, true>(njobs, lds_cells, jobs, job_offset, progs, steps, ops, x, cap, \
                                                   ord_mask, st)                                                  \
                          : leaf2_launch<CC, false>(njobs, lds_cells, jobs, job_offset, progs, steps, ops, x, cap, \
                                                    ord_mask, st);
    switch (W) {
        TFT_LEAF2_CASE(16)
        TFT_LEAF2_CASE(32)
        default: return hipErrorInvalidValue;
    }
#undef TFT_LEAF2_CASE
}

}  // namespace tft
