// Host-side launchers for R = (Z/mZ)[y]/(y^K+1), theta = y (Sect. 5.2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "desc.hpp"

namespace tft {

hipError_t launch_nega_leaf(uint32_t K, uint64_t m, uint32_t nwaves, uint32_t njobs, uint32_t lds_cells,
                            const Job *jobs, uint32_t job_offset, const LeafProg *progs, const LeafStep *steps,
                            const LeafOp *ops, uint64_t *x, uint32_t ord_mask, hipStream_t st);

// c_i = a_i b_i 2^-scale_log2 (negacyclic product of K coefficients mod m) for i < n.
hipError_t launch_nega_pointwise(uint32_t K, uint64_t m, uint64_t n, const uint64_t *a, const uint64_t *b,
                                 uint64_t *c, uint32_t scale_log2, hipStream_t st);

// Cut len coefficients into pieces of K/2 placed in the low halves of cells [0, pieces).
hipError_t launch_nega_pack(uint32_t K, const uint64_t *coef, uint64_t len, uint64_t *x, uint64_t pieces,
                            hipStream_t st);

// Overlap-add cells [0, pieces) at offsets p*K/2 into out_len coefficients mod m.
hipError_t launch_nega_unpack(uint32_t K, uint64_t m, const uint64_t *x, uint64_t pieces, uint64_t *out,
                              uint64_t out_len, hipStream_t st);

}  // namespace tft
