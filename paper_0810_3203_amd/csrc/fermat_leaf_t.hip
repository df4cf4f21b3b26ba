// Leaf kernels for cell arrays in the transposed (LDS order) layout.
#include "fermat_leaf.hpp"

namespace tft {

hipError_t launch_fermat_leaf_trans(uint32_t W, uint32_t nwaves, uint32_t njobs, uint32_t lds_cells, const Job *jobs,
                              uint32_t job_offset, const LeafProg *progs, const LeafStep *steps, const LeafOp *ops,
                              uint32_t *x, uint64_t cap, uint32_t ord_mask, uint32_t opmask, hipStream_t st) {
    if (njobs == 0) return hipSuccess;
    TFT_FERMAT_DISPATCH(W, LeafLaunch<true>::run, nwaves, njobs, lds_cells, jobs, job_offset, progs, steps, ops, x, cap,
                        ord_mask, opmask, st)
}

}  // namespace tft
