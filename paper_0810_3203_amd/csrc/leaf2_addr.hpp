// Address arithmetic of the persistent leaf executor (fermat_leaf2.hpp), kept
// free of device code so that a host program can check every address the
// kernel forms against its LDS allocation and its job's cells.
//
// LDS of one workgroup (dword offsets): [0, W) holds the top words of the leaf
// cells; cell i occupies [W + i W, W + (i+1) W), limb k of a cell at
// (k mod C) 64 + k / C (lane l's limb j at j 64 + l), W = 64 C.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define TFT_HD __host__ __device__ __forceinline__
#else
#define TFT_HD inline
#endif

namespace tft {
namespace lf2 {

constexpr int kQuadsPerThread = 16;
constexpr uint32_t kThreads = 512;

TFT_HD constexpr uint32_t cell_base(uint32_t W, uint32_t i) { return W + i * W; }
TFT_HD constexpr uint32_t lds_dwords(uint32_t W, uint32_t cells) { return W * (cells + 1u); }
// LDS offset of limb k inside a cell
TFT_HD constexpr uint32_t limb_pos(uint32_t C, uint32_t k) { return (k % C) * 64u + k / C; }

// Quad r (4 limbs) of a cell.  Plain global order: limbs 4m..4m+3 of lane l,
// l = r mod 64, m = r / 64, at global dword l C + 4m, LDS rows 4m..4m+3 of
// column l.  Transposed global order (the LDS order): dwords 4r..4r+3 in both.
TFT_HD constexpr uint32_t quad_lane(uint32_t r) { return r % 64u; }
TFT_HD constexpr uint32_t quad_m(uint32_t r) { return r / 64u; }
TFT_HD constexpr uint32_t plain_quad_offset(uint32_t C, uint32_t r) { return quad_lane(r) * C + 4u * quad_m(r); }

// Thread tid moves quads q = tid + 512 i (i < 16) of a job's cell list: cell
// c0 + i K, quad r of it, K = 512 / (W/4), c0 = tid / (W/4), r = tid mod (W/4).
TFT_HD constexpr uint32_t quad_cells_per_sweep(uint32_t C) { return kThreads / (16u * C); }
TFT_HD constexpr uint32_t quad_c0(uint32_t C, uint32_t tid) { return tid / (16u * C); }
TFT_HD constexpr uint32_t quad_r(uint32_t C, uint32_t tid) { return tid % (16u * C); }
TFT_HD constexpr uint32_t quad_loff(uint32_t C, bool tr, uint32_t tid) {
    return tr ? 4u * quad_r(C, tid) : 4u * quad_m(quad_r(C, tid)) * 64u + quad_lane(quad_r(C, tid));
}
TFT_HD constexpr uint32_t quad_goff(uint32_t C, bool tr, uint32_t tid) {
    return tr ? 4u * quad_r(C, tid) : plain_quad_offset(C, quad_r(C, tid));
}
// LDS dword offsets of the 4 words of the thread's quad i: base, base + step, ...
TFT_HD constexpr uint32_t quad_lds(uint32_t C, bool tr, uint32_t tid, uint32_t i) {
    return cell_base(64u * C, quad_c0(C, tid) + i * quad_cells_per_sweep(C)) + quad_loff(C, tr, tid);
}
TFT_HD constexpr uint32_t quad_lds_step(bool tr) { return tr ? 1u : 64u; }

// Rotated read of lane l (multiplication by 2^t, qp = ceil(t / 32) limbs):
// word i = 0..C is limb (l C - qp + i) mod W, read at base A + 64 i while
// row0 + i < C, else at base B + 64 i; B = e + row0 64 + col1 - 64 C is not
// negative because every cell starts at e >= W.
TFT_HD constexpr uint32_t rot_row0(uint32_t C, uint32_t qp) { return (0u - qp) & (C - 1u); }
TFT_HD constexpr uint32_t rot_col0(uint32_t C, uint32_t l, uint32_t qp) { return ((l * C - qp) & (64u * C - 1u)) / C; }
TFT_HD constexpr uint32_t rot_base_a(uint32_t C, uint32_t e, uint32_t l, uint32_t qp) {
    return e + rot_row0(C, qp) * 64u + rot_col0(C, l, qp);
}
TFT_HD constexpr uint32_t rot_base_b(uint32_t C, uint32_t e, uint32_t l, uint32_t qp) {
    return e + rot_row0(C, qp) * 64u + ((rot_col0(C, l, qp) + 1u) & 63u) - 64u * C;
}
TFT_HD constexpr uint32_t rot_word(uint32_t C, uint32_t e, uint32_t l, uint32_t qp, uint32_t i) {
    return (i + rot_row0(C, qp) < C ? rot_base_a(C, e, l, qp) : rot_base_b(C, e, l, qp)) + 64u * i;
}

}  // namespace lf2
}  // namespace tft
