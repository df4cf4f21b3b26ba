// Plain descriptors shared by the host planner and the leaf kernels.
//
// A transform runs as a sequence of passes (kernel launches).  Each pass holds
// independent leaf jobs; a leaf job is one sub-transform of Alg. 1 or Alg. 2
// small enough for one workgroup's LDS: it names the cells it owns in the
// global array (base, stride), the leaf program to run and the concrete twist
// exponent s of its zeta.  A leaf program is a list of steps separated by
// workgroup barriers; each step is a list of independent base-case operations
// (the L = 2 cases of Alg. 1 and Alg. 2) on cells of the leaf.
#pragma once
#include <stdint.h>

namespace tft {

// Base cases of Alg. 1 (TFT) and Alg. 2 (ITFT) at L = 2.
enum BaseOp : uint32_t {
    OP_NONE = 0,
    OP_T22 = 1,     // TFT  z=2 n=2: (x0, x1) <- (x0 + x1, zeta (x0 - x1))
    OP_T21 = 2,     // TFT  z=1 n=2: x1 <- zeta x0
    OP_T12 = 3,     // TFT  z=2 n=1: x0 <- x0 + x1
    OP_I2 = 4,      // ITFT n=2:         (x0, x1) <- (x0 + x1/zeta, x0 - x1/zeta)
    OP_I1F1Z2 = 5,  // ITFT n=1 f=1 z=2: (x0, x1) <- (2 x0 - x1, zeta (x0 - x1))
    OP_I1F1Z1 = 6,  // ITFT n=1 f=1 z=1: (x0, x1) <- (2 x0, zeta x0)
    OP_I1F0Z2 = 7,  // ITFT n=1 f=0 z=2: x0 <- 2 x0 - x1
    OP_I1F0Z1 = 8,  // ITFT n=1 f=0 z=1: x0 <- 2 x0
    OP_I0Z2 = 9,    // ITFT n=0 z=2:     x0 <- (x0 + x1) / 2
    OP_I0Z1 = 10,   // ITFT n=0 z=1:     x0 <- x0 / 2
};

// w0 = opcode | i0 << 4 | i1 << 18 ; w1 = b | alog << 28 (b < 2^28: ord(theta)
// up to 2^27 for Z/pZ; alog, the depth inside a leaf, < 16).
// The operation's twist exponent is (s * 2^alog + b) mod ord(theta), s being the job's.
constexpr uint32_t kOpAlogShift = 28;
constexpr uint32_t kOpBMask = (1u << kOpAlogShift) - 1u;
struct LeafOp {
    uint32_t w0;
    uint32_t w1;
};

struct LeafStep {
    uint32_t op_begin;
    uint32_t op_count;
};

struct LeafProg {
    uint32_t step_begin;
    uint32_t step_count;
    uint32_t len;
    uint32_t max_ops;  // largest op_count over the program's steps
};

struct Job {
    uint64_t base;    // global cell index of leaf cell 0
    uint64_t stride;  // global cell distance between leaf cells
    uint32_t prog;    // program index
    uint32_t s;       // twist exponent of this sub-transform's zeta (mod ord)
    uint32_t nload;   // leaf cells [0, nload) are inputs
    uint32_t nstore;  // leaf cells [0, nstore) are outputs
};

static_assert(sizeof(Job) == 32, "Job layout");

// One operand of a Schoenhage-Strassen product: len coefficients of climbs
// limbs, k per cell in slots of ws limbs, written to cells [cell0, cell0 + z).
struct PackDesc {
    const uint32_t *coef;
    uint64_t len;
    uint64_t cell0;
    uint64_t z;
    uint32_t climbs;
    uint32_t k;
    uint32_t ws;
    uint32_t pad;
};

// One product: len_out coefficients of olimbs limbs from the ncells cells at cell0.
struct UnpackDesc {
    uint32_t *out;
    uint64_t len_out;
    uint64_t cell0;
    uint64_t ncells;
    uint32_t olimbs;
    uint32_t k;
    uint32_t ws;
    uint32_t pad;
};

constexpr uint32_t op_code(const LeafOp &o) { return o.w0 & 15u; }
constexpr uint32_t op_i0(const LeafOp &o) { return (o.w0 >> 4) & 16383u; }
constexpr uint32_t op_i1(const LeafOp &o) { return (o.w0 >> 18) & 16383u; }
constexpr uint32_t op_b(const LeafOp &o) { return o.w1 & kOpBMask; }
constexpr uint32_t op_alog(const LeafOp &o) { return o.w1 >> kOpAlogShift; }

}  // namespace tft
