// Host check of every address the persistent leaf executor forms (the
// functions of leaf2_addr.hpp that the kernel itself calls): for each element
// size, cell layout and leaf size the kernel accepts, the quads each thread
// moves, the rotated reads of every lane, rotation and word, and the ripple
// and store positions all lie inside the workgroup's LDS allocation and the
// job's cells, and the copies cover each cell exactly once.  Prints one line
// per failure and exits non-zero if there was any.
//
// It also evaluates the base of the rotated reads that the earlier executor
// formed without a guard block (cells from LDS offset 0): that base lies below
// the allocation for the first cell, the condition that, through a 64-bit
// generic (flat) address, leaves the LDS aperture.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "leaf2_addr.hpp"

using namespace tft::lf2;

static int failures = 0;
#define CHECK(cond, ...)                      \
    do {                                      \
        if (!(cond)) {                        \
            if (failures < 20) {              \
                std::printf("FAIL: " __VA_ARGS__); \
                std::printf("\n");            \
            }                                 \
            failures++;                       \
        }                                     \
    } while (0)

static uint32_t max_cells(uint32_t C) {
    const uint32_t W = 64u * C;
    uint32_t by_quads = (uint32_t)kQuadsPerThread * kThreads / (W / 4u);
    uint32_t by_lds = 160u * 1024u / (4u * W) - 1u;
    uint32_t m = by_quads < by_lds ? by_quads : by_lds;
    uint32_t p = 1;
    while (2 * p <= m) p *= 2;
    return p;  // the planner's leaves are powers of two
}

int main() {
    long checks = 0;
    for (uint32_t C = 4; C <= 32; C *= 2) {
        const uint32_t W = 64u * C;
        const uint32_t mc = max_cells(C);
        CHECK(lds_dwords(W, mc) * 4u <= 160u * 1024u, "C=%u: LDS of %u cells exceeds 160 KB", C, mc);
        CHECK(mc <= W, "C=%u: %u top words do not fit the guard block", C, mc);
        for (int tr = 0; tr < 2; ++tr) {
            for (uint32_t nc = 1; nc <= mc; ++nc) {
                std::vector<uint8_t> lds_hit(lds_dwords(W, nc), 0);
                std::vector<uint8_t> glob_hit((size_t)nc * W, 0);
                for (uint32_t tid = 0; tid < kThreads; ++tid) {
                    for (uint32_t i = 0; i < (uint32_t)kQuadsPerThread; ++i) {
                        const uint32_t cell = quad_c0(C, tid) + i * quad_cells_per_sweep(C);
                        if (cell >= nc) continue;
                        const uint32_t a = quad_lds(C, tr, tid, i);
                        const uint32_t g = quad_goff(C, tr, tid);
                        for (uint32_t w = 0; w < 4; ++w) {
                            const uint32_t la = a + w * quad_lds_step(tr);
                            const uint32_t gk = g + w;  // dword of the global cell
                            ++checks;
                            CHECK(la >= cell_base(W, cell) && la < cell_base(W, cell) + W,
                                  "C=%u tr=%d nc=%u tid=%u i=%u: LDS word %u outside cell %u", C, tr, nc, tid, i, la,
                                  cell);
                            CHECK(gk < W, "C=%u tr=%d tid=%u: global dword %u outside the cell", C, tr, tid, gk);
                            // the LDS position must hold the limb the global dword holds
                            const uint32_t want = tr ? cell_base(W, cell) + gk : cell_base(W, cell) + limb_pos(C, gk);
                            CHECK(la == want, "C=%u tr=%d tid=%u i=%u: quad word %u at LDS %u, limb wants %u", C, tr,
                                  tid, i, w, la, want);
                            if (la < lds_hit.size()) lds_hit[la]++;
                            if (gk < W) glob_hit[(size_t)cell * W + gk]++;
                        }
                    }
                }
                for (uint32_t d = W; d < lds_dwords(W, nc); ++d)
                    CHECK(lds_hit[d] == 1, "C=%u tr=%d nc=%u: LDS dword %u written %u times", C, tr, nc, d,
                          lds_hit[d]);
                for (size_t d = 0; d < glob_hit.size(); ++d)
                    CHECK(glob_hit[d] == 1, "C=%u tr=%d nc=%u: global dword %zu moved %u times", C, tr, nc, d,
                          glob_hit[d]);
            }
        }
        // rotated reads, first and last cell of the largest leaf
        for (uint32_t cell : {0u, mc - 1u}) {
            const uint32_t e = cell_base(W, cell);
            for (uint32_t qp = 0; qp <= W; ++qp) {
                const int64_t row0 = rot_row0(C, qp);
                for (uint32_t l = 0; l < 64; ++l) {
                    const int64_t col1 = (rot_col0(C, l, qp) + 1u) & 63u;
                    CHECK((int64_t)e + row0 * 64 + col1 - 64 * (int64_t)C >= 0,
                          "C=%u cell=%u qp=%u lane=%u: second base below the allocation", C, cell, qp, l);
                    for (uint32_t i = 0; i <= C; ++i) {
                        ++checks;
                        const uint32_t a = rot_word(C, e, l, qp, i);
                        const uint32_t k = (l * C + W - (qp % W) + i) % W;
                        CHECK(a == e + limb_pos(C, k), "C=%u qp=%u lane=%u word=%u: address %u, limb %u at %u", C,
                              qp, l, i, a, k, e + limb_pos(C, k));
                    }
                }
            }
        }
        // ripple and store positions: every limb of every cell
        for (uint32_t k = 0; k < W; ++k) CHECK(limb_pos(C, k) < W, "C=%u: limb %u outside the cell", C, k);
    }
    // the earlier executor's rotated-read base, cells from offset 0 (no guard block)
    int below = 0;
    for (uint32_t C = 4; C <= 32; C *= 2)
        for (uint32_t qp = 0; qp <= 64u * C; ++qp)
            for (uint32_t l = 0; l < 64; ++l) {
                const int64_t b = (int64_t)rot_row0(C, qp) * 64 + ((rot_col0(C, l, qp) + 1u) & 63u) - 64 * (int64_t)C;
                if (b < 0) below++;
            }
    std::printf("checks %ld failures %d unguarded_negative_bases %d\n", checks, failures, below);
    return failures ? 1 : 0;
}
