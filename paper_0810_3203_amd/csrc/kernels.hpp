// Host-side launchers of the HIP kernels (one instantiation per element size).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "desc.hpp"

namespace tft {

// Cell layouts in global memory: plain (limb k of a cell at offset k, the ABI
// layout) or transposed (limb k at (k mod C) 64 + k / C for W = 64 C >= 128, the
// order a leaf keeps in LDS; used for the cell arrays inside products).  For
// W <= 64 both are the same.

// Leaf workgroups for one pass of a Fermat-ring transform.
// opmask: BaseOp bits the pass's programs use; selects a kernel compiled for that set of base cases.
hipError_t launch_fermat_leaf(uint32_t W, uint32_t nwaves, uint32_t njobs, uint32_t lds_cells, const Job *jobs,
                              uint32_t job_offset, const LeafProg *progs, const LeafStep *steps, const LeafOp *ops,
                              uint32_t *x, uint64_t cap, uint32_t ord_mask, uint32_t opmask, bool transposed,
                              hipStream_t st);
hipError_t launch_fermat_leaf_plain(uint32_t W, uint32_t nwaves, uint32_t njobs, uint32_t lds_cells, const Job *jobs,
                                    uint32_t job_offset, const LeafProg *progs, const LeafStep *steps,
                                    const LeafOp *ops, uint32_t *x, uint64_t cap, uint32_t ord_mask, uint32_t opmask,
                                    hipStream_t st);
hipError_t launch_fermat_leaf_trans(uint32_t W, uint32_t nwaves, uint32_t njobs, uint32_t lds_cells, const Job *jobs,
                                    uint32_t job_offset, const LeafProg *progs, const LeafStep *steps,
                                    const LeafOp *ops, uint32_t *x, uint64_t cap, uint32_t ord_mask, uint32_t opmask,
                                    hipStream_t st);

// Persistent leaf executor (fermat_leaf2.hpp), used for W = 1024 and 2048: 512
// threads per workgroup, one workgroup per compute unit, the next job's cells
// loaded into registers while the current job runs.
bool fermat_leaf2_supported(uint32_t W);
hipError_t launch_fermat_leaf2(uint32_t W, uint32_t njobs, uint32_t lds_cells, const Job *jobs, uint32_t job_offset,
                               const LeafProg *progs, const LeafStep *steps, const LeafOp *ops, uint32_t *x,
                               uint64_t cap, uint32_t ord_mask, uint32_t opmask, bool transposed, hipStream_t st);

// Single base cases of the persistent executor, one wave each (self-test of its arithmetic).
hipError_t launch_base_case_probe(uint32_t W, uint32_t ncases, const uint32_t *in, uint32_t *out, hipStream_t st);

// c_i = a_i b_i 2^scale_e (scale_e = -scale_log2 mod 2N) for i < n, cell arrays of capacity cap.
hipError_t launch_fermat_pointwise(uint32_t W, uint64_t n, const uint32_t *a, const uint32_t *b, uint32_t *c,
                                   uint64_t cap, uint32_t scale_e, bool transposed, hipStream_t st);

// Pointwise products over an item list on one cell array (see fermat_pointwise_items_kernel).
hipError_t launch_fermat_pointwise_items(uint32_t W, uint64_t nitems, uint32_t *x, uint64_t cap, const uint4 *items,
                                         bool transposed, hipStream_t st);

// Coefficients -> cells, one descriptor per operand: a device array of ndesc
// descriptors, or (descs == nullptr, ndesc == 1) the descriptor inl passed by value.
hipError_t launch_fermat_pack(uint32_t W, const PackDesc *descs, uint32_t ndesc, const PackDesc &inl, uint64_t max_z,
                              uint32_t *x, uint64_t cap, bool transposed, hipStream_t st);

// Cells -> coefficients, one descriptor per product (device array or inl as above);
// bundled = the descriptors have k > 1 (all of one launch alike).
hipError_t launch_fermat_unpack(uint32_t W, const UnpackDesc *descs, uint32_t ndesc, const UnpackDesc &inl,
                                uint64_t max_len, uint32_t max_olimbs, bool bundled, const uint32_t *x, uint64_t cap,
                                bool transposed, hipStream_t st);

// Leaf pass over R = Z/pZ (prime.hip): jobs packed per workgroup, optw the
// per-op twiddle table (Montgomery theta^b, theta^-b for the inverse
// butterfly), zw = entries of each job's twist table (every op's alog < zw).
hipError_t launch_zp_leaf(uint32_t njobs, uint32_t max_len, uint32_t max_ops, const Job *jobs, uint32_t job_begin,
                          const LeafProg *progs, const LeafStep *steps, const LeafOp *ops, const uint32_t *optw,
                          uint32_t *x, uint32_t zw, hipStream_t st);
// c_i = a_i b_i 2^-scale_log2 in Z/pZ for i < n.
hipError_t launch_zp_pointwise(uint64_t n, const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t scale_log2,
                               hipStream_t st);

// Largest LDS bytes one workgroup may use.
uint32_t lds_budget_bytes();

// Records a failed HIP call for tft_last_error; returns TFT_E_DEVICE.
int device_error(hipError_t e, const char *where);

// LDS bytes of one Fermat cell inside a leaf workgroup (limbs plus top word).
uint32_t fermat_lds_cell_bytes(uint32_t W);

}  // namespace tft
