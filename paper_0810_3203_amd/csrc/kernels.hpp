// Host-side launchers of the HIP kernels (one instantiation per element size).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "desc.hpp"

namespace tft {

// Leaf workgroups for one pass of a Fermat-ring transform.
hipError_t launch_fermat_leaf(uint32_t W, uint32_t nwaves, uint32_t njobs, uint32_t lds_cells, const Job *jobs,
                              uint32_t job_offset, const LeafProg *progs, const LeafStep *steps, const LeafOp *ops,
                              uint32_t *x, uint64_t cap, uint32_t ord_mask, hipStream_t st);

// c_i = a_i b_i 2^scale_e (scale_e = -scale_log2 mod 2N) for i < n, cell arrays of capacity cap.
hipError_t launch_fermat_pointwise(uint32_t W, uint64_t n, const uint32_t *a, const uint32_t *b, uint32_t *c,
                                   uint64_t cap, uint32_t scale_e, hipStream_t st);

// Coefficients (climbs limbs each) -> cells [0, count) of a cell array of capacity cap.
hipError_t launch_fermat_pack(uint32_t W, const uint32_t *coef, uint64_t count, uint32_t climbs, uint32_t *x,
                              uint64_t cap, hipStream_t st);

// Cells [0, count) -> coefficients of olimbs limbs (low limbs of the canonical residue).
hipError_t launch_fermat_unpack(uint32_t W, const uint32_t *x, uint64_t cap, uint64_t count, uint32_t *out,
                                uint32_t olimbs, hipStream_t st);

// Largest LDS bytes one workgroup may use.
uint32_t lds_budget_bytes();

// LDS bytes of one Fermat cell inside a leaf workgroup (padded chunk layout plus top word).
uint32_t fermat_lds_cell_bytes(uint32_t W);

}  // namespace tft
