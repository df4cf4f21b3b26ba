// Host planner: expands Alg. 1 (CacheFriendlyTFT, Sect. 3) and Alg. 2
// (CacheFriendlyITFT, Sect. 4) into passes of leaf jobs and leaf programs.
//
// Above the leaf size the planner follows the algorithms' recursion exactly,
// with the split L1 = 2^floor(l/2), L2 = 2^ceil(l/2) (or a chosen top split):
// every recursive call on a column c_u or a row r_u becomes a sub-plan on the
// strided view of that column or row.  Sub-transforms that fit one
// workgroup's LDS become leaf jobs; inside a leaf the same algorithms run with
// the split L1 = 2 (van der Hoeven's form, the paper's remark after the split
// rule), flattened into steps of independent base cases.  Any split computes
// the same outputs (eqs. (b-cols) and (b-rows) hold for every l1 + l2 = l).
#pragma once
#include <map>
#include <stdint.h>
#include <tuple>
#include <vector>

#include "desc.hpp"

namespace tft {

constexpr uint32_t kSplitDC = 0xFFFFFFFFu;  // TFT_SPLIT_DC of the C interface

struct PassDesc {
    uint32_t job_begin;
    uint32_t job_count;
    uint32_t max_len;  // largest leaf length among the pass's jobs
    uint32_t max_ops;  // largest step width among the pass's programs
    uint32_t opmask;   // bit c set if a job of the pass runs base case c (BaseOp)
};

struct Schedule {
    uint32_t direction = 0;  // 0 TFT, 1 ITFT
    uint32_t ord = 0;        // order of theta (a power of two here)
    uint32_t leaf_log2 = 0;
    uint32_t top_l1 = 0;
    std::vector<PassDesc> passes;
    std::vector<Job> jobs;
    std::vector<LeafProg> progs;
    std::vector<LeafStep> steps;
    std::vector<LeafOp> ops;
    std::vector<uint32_t> prog_base_cases;  // base cases per program (no-ops included)
    std::vector<uint32_t> prog_opmask;      // BaseOp bits used per program
    uint64_t base_cases = 0;
};

// Build the schedule of TFT(L, theta^s, z, n) (direction 0) or
// ITFT(L, theta^s, z, n, f) (direction 1) on an array of L = 2^l cells.
// ord = order of theta; leaf_log2 = largest leaf (>= 1); top_l1 = 0 for the
// paper's split, kSplitDC for L1 = 2 at every level above the leaf (van der
// Hoeven's divide-and-conquer order).  Below the top, sub-transforms larger
// than a leaf are split leaf-major (columns one whole leaf where two leaves
// cover them) or, with balanced, into the fewest passes as evenly as they
// allow (for small cells, where a pass of tiny jobs would be all overhead).
// Arguments must already be valid.
Schedule build_schedule(uint32_t direction, uint32_t l, uint32_t ord, uint64_t s, uint64_t z, uint64_t n, uint32_t f,
                        uint32_t leaf_log2, uint32_t top_l1, bool balanced = false);

// Number of passes build_schedule gives for the same arguments, from the
// recursion alone (no jobs are built): the column and row sub-plans of one
// level that share a shape take the same passes, so only the distinct shapes
// of each level are followed.
uint32_t schedule_pass_count(uint32_t direction, uint32_t l, uint64_t z, uint64_t n, uint32_t f, uint32_t leaf_log2,
                             uint32_t top_l1, bool balanced = false);

}  // namespace tft
