// Host run of the leaf executor's wave-level arithmetic (fermat_leaf2_ops.hpp,
// the code the kernel itself runs) under a lockstep emulation of one
// wavefront: 64 threads are the lanes, and every cross-lane operation (lane
// masks, reads of one lane's value, the LDS hand-offs marked wave_sync) waits
// for all of them.  For each case it prints the inputs and outputs of one
// base case of Alg. 1 / Alg. 2 on two cells in LDS; tests/test_leaf2_emu.py
// checks them with Python integers.
//
// usage: leaf2_ops_emu <C> <cases> <seed>
#include <atomic>
#include <array>
#include <barrier>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <random>
#include <thread>
#include <vector>

namespace tft {
namespace lf2 {
namespace emu {
struct Wave {
    std::barrier<> bar{64};
    std::atomic<uint64_t> acc{0};
    uint32_t vals[64];
};
inline Wave *g_wave = nullptr;
inline thread_local uint32_t t_lane = 0;
inline uint32_t lane() { return t_lane; }
inline void sync() { g_wave->bar.arrive_and_wait(); }
inline uint64_t ballot(bool p) {
    Wave &w = *g_wave;
    w.bar.arrive_and_wait();
    if (p) w.acc.fetch_or(1ull << t_lane);
    w.bar.arrive_and_wait();
    const uint64_t r = w.acc.load();
    w.bar.arrive_and_wait();
    if (t_lane == 0) w.acc.store(0);
    return r;
}
inline uint32_t readlane(uint32_t v, int src) {
    Wave &w = *g_wave;
    w.bar.arrive_and_wait();
    w.vals[t_lane] = v;
    w.bar.arrive_and_wait();
    const uint32_t r = w.vals[src];
    w.bar.arrive_and_wait();
    return r;
}
}  // namespace emu
}  // namespace lf2
}  // namespace tft

#define TFT_WAVE_EMU 1
#include "fermat_leaf2_ops.hpp"

using namespace tft;
using namespace tft::lf2;

struct Case {
    uint32_t code, s;
    std::vector<uint32_t> x[2];
    uint32_t top[2];
};

template <int C>
static void run(int ncases, uint64_t seed) {
    constexpr uint32_t W = 64u * C, N = 32u * W;
    std::mt19937_64 rng(seed);
    auto rnd = [&]() { return (uint32_t)rng(); };
    // operands: random, zero, one, 2^N (top), 2^N - 1, sparse halves, chunk-aligned
    // runs of zeros and ones, values with long zero runs below
    auto make = [&](int kind, std::vector<uint32_t> &v, uint32_t &top) {
        v.assign(W, 0u);
        top = 0;
        switch (kind) {
            case 0: for (auto &w : v) w = rnd(); break;
            case 1: break;
            case 2: v[0] = 1; break;
            case 3: top = 1; break;
            case 4: for (auto &w : v) w = ~0u; break;
            case 5: for (uint32_t k = 0; k < W / 2; ++k) v[k] = rnd(); break;
            case 6: for (uint32_t k = W / 2; k < W; ++k) v[k] = rnd(); break;
            case 7:  // chunks all zero or all ones, random lanes
                for (uint32_t ln = 0; ln < 64; ++ln) {
                    const uint32_t f = (rnd() & 1) ? ~0u : 0u;
                    for (uint32_t j = 0; j < C; ++j) v[ln * C + j] = f;
                }
                v[rnd() % W] = rnd();
                break;
            case 8: v[rnd() % W] = rnd(); break;  // one limb
            case 9:  // ones with a random cut
                for (uint32_t k = rnd() % W; k < W; ++k) v[k] = ~0u;
                break;
            default: for (uint32_t k = rnd() % W; k < W; ++k) v[k] = rnd(); break;
        }
    };
    std::vector<Case> cases(ncases);
    const uint32_t codes[] = {OP_T22, OP_T21, OP_T12, OP_I2, OP_I1F1Z2, OP_I1F1Z1, OP_I1F0Z2, OP_I1F0Z1, OP_I0Z2, OP_I0Z1};
    const uint32_t special[] = {0u, 1u, 31u, 32u, 33u, 32u * C - 1u, 32u * C, 32u * C + 1u, N - 1u, N, N + 1u, 2 * N - 1u,
                                N / 2, 3 * N / 2};
    for (int i = 0; i < ncases; ++i) {
        Case &c = cases[i];
        c.code = codes[i % 10];
        c.s = (i / 10) % 3 == 0 ? special[(i / 10 / 3) % 14] : (uint32_t)(rng() % (2 * N));
        // half of the cases take both operands of one kind (sparse pairs)
        const int k0 = (int)(rng() % 11);
        make(k0, c.x[0], c.top[0]);
        make((rng() & 1) ? k0 : (int)(rng() % 11), c.x[1], c.top[1]);
    }
    std::vector<uint32_t> sm(lds_dwords(W, 2), 0u);
    std::vector<std::vector<uint32_t>> outs(ncases);
    std::vector<std::array<uint32_t, 2>> otop(ncases);
    emu::Wave wave;
    emu::g_wave = &wave;
    auto body = [&](uint32_t ln) {
        emu::t_lane = ln;
        const Big<C> ar;
        for (int i = 0; i < ncases; ++i) {
            const Case &c = cases[i];
            if (ln == 0) {
                for (int e = 0; e < 2; ++e) {
                    for (uint32_t k = 0; k < W; ++k) sm[cell_base(W, e) + limb_pos(C, k)] = c.x[e][k];
                    sm[e] = c.top[e];
                }
            }
            emu::sync();
            LeafOp o{c.code | (0u << 4) | (1u << 18), 0u};
            base_case<C>(ar, sm.data(), o, c.s, 2 * N - 1);
            emu::sync();
            if (ln == 0) {
                outs[i].resize(2 * W);
                for (int e = 0; e < 2; ++e) {
                    for (uint32_t k = 0; k < W; ++k) outs[i][e * W + k] = sm[cell_base(W, e) + limb_pos(C, k)];
                    otop[i][e] = sm[e];
                }
            }
            emu::sync();
        }
    };
    std::vector<std::thread> th;
    for (uint32_t ln = 0; ln < 64; ++ln) th.emplace_back(body, ln);
    for (auto &t : th) t.join();
    auto hex = [&](const uint32_t *v) {
        std::string s;
        char b[9];
        for (int k = (int)W - 1; k >= 0; --k) {
            std::snprintf(b, sizeof b, "%08x", v[k]);
            s += b;
        }
        return s;
    };
    for (int i = 0; i < ncases; ++i) {
        const Case &c = cases[i];
        std::printf("%d %u %u %s %u %s %u %s %u %s %u\n", C, c.code, c.s, hex(c.x[0].data()).c_str(), c.top[0],
                    hex(c.x[1].data()).c_str(), c.top[1], hex(outs[i].data()).c_str(), otop[i][0],
                    hex(outs[i].data() + W).c_str(), otop[i][1]);
    }
}

// Plan mode: reads "C cap ord nprogs nsteps nops njobs" then the programs
// (step_begin step_count len), steps (op_begin op_count), ops (w0 w1), the jobs
// in pass order (base stride prog s nload nstore, one pass after another: each
// job reads the array as the previous passes left it), then cap cells of W
// limbs and a top each (hex, most significant limb first); runs every job on
// one emulated wave and prints the cells.
template <int C>
static int run_plan() {
    constexpr uint32_t W = 64u * C;
    uint64_t cap;
    uint32_t ord, np, ns, no, nj;
    if (std::scanf("%lu %u %u %u %u %u", &cap, &ord, &np, &ns, &no, &nj) != 6) return 3;
    std::vector<LeafProg> progs(np);
    std::vector<LeafStep> steps(ns);
    std::vector<LeafOp> ops(no);
    std::vector<Job> jobs(nj);
    for (auto &p : progs) std::scanf("%u %u %u", &p.step_begin, &p.step_count, &p.len);
    for (auto &t : steps) std::scanf("%u %u", &t.op_begin, &t.op_count);
    for (auto &o : ops) std::scanf("%u %u", &o.w0, &o.w1);
    for (auto &j : jobs) std::scanf("%lu %lu %u %u %u %u", &j.base, &j.stride, &j.prog, &j.s, &j.nload, &j.nstore);
    std::vector<uint32_t> x(cap * W), tops(cap);
    std::vector<char> buf(8 * W + 16);
    for (uint64_t i = 0; i < cap; ++i) {
        std::scanf("%s %u", buf.data(), &tops[i]);
        for (uint32_t k = 0; k < W; ++k) {
            char t[9];
            std::memcpy(t, buf.data() + 8 * (W - 1 - k), 8);
            t[8] = 0;
            x[i * W + k] = (uint32_t)std::strtoul(t, nullptr, 16);
        }
    }
    uint32_t maxlen = 1;
    for (auto &p : progs) maxlen = p.len > maxlen ? p.len : maxlen;
    std::vector<uint32_t> sm(lds_dwords(W, maxlen), 0xDEADBEEFu);
    emu::Wave wave;
    emu::g_wave = &wave;
    auto body = [&](uint32_t ln) {
        emu::t_lane = ln;
        const Big<C> ar;
        for (const Job &J : jobs) {
            if (ln == 0) {
                for (uint32_t c = 0; c < J.nload; ++c) {
                    const uint64_t g = J.base + c * J.stride;
                    for (uint32_t k = 0; k < W; ++k) sm[cell_base(W, c) + limb_pos(C, k)] = x[g * W + k];
                    sm[c] = tops[g];
                }
            }
            emu::sync();
            const LeafProg &P = progs[J.prog];
            for (uint32_t st = 0; st < P.step_count; ++st) {
                const LeafStep &LS = steps[P.step_begin + st];
                for (uint32_t j = 0; j < LS.op_count; ++j) base_case<C>(ar, sm.data(), ops[LS.op_begin + j], J.s, ord - 1);
            }
            emu::sync();
            if (ln == 0) {
                for (uint32_t c = 0; c < J.nstore; ++c) {
                    const uint64_t g = J.base + c * J.stride;
                    for (uint32_t k = 0; k < W; ++k) x[g * W + k] = sm[cell_base(W, c) + limb_pos(C, k)];
                    tops[g] = sm[c];
                }
            }
            emu::sync();
        }
    };
    std::vector<std::thread> th;
    for (uint32_t ln = 0; ln < 64; ++ln) th.emplace_back(body, ln);
    for (auto &t : th) t.join();
    for (uint64_t i = 0; i < cap; ++i) {
        for (int k = (int)W - 1; k >= 0; --k) std::printf("%08x", x[i * W + k]);
        std::printf(" %u\n", tops[i]);
    }
    return 0;
}

// Record mode: reads lines "code s top0 top1 x0hex x1hex" (most significant
// limb first) and prints "top0' top1' x0'hex x1'hex" for each.
template <int C>
static int run_records() {
    constexpr uint32_t W = 64u * C, N = 32u * W;
    std::vector<Case> cases;
    std::vector<char> b0(8 * W + 16), b1(8 * W + 16);
    uint32_t code, sx, t0, t1;
    auto parse = [&](const char *h, std::vector<uint32_t> &v) {
        v.assign(W, 0u);
        for (uint32_t k = 0; k < W; ++k) {
            char t[9];
            std::memcpy(t, h + 8 * (W - 1 - k), 8);
            t[8] = 0;
            v[k] = (uint32_t)std::strtoul(t, nullptr, 16);
        }
    };
    while (std::scanf("%u %u %u %u %s %s", &code, &sx, &t0, &t1, b0.data(), b1.data()) == 6) {
        Case c;
        c.code = code;
        c.s = sx;
        c.top[0] = t0;
        c.top[1] = t1;
        parse(b0.data(), c.x[0]);
        parse(b1.data(), c.x[1]);
        cases.push_back(c);
    }
    const int n = (int)cases.size();
    std::vector<uint32_t> sm(lds_dwords(W, 2), 0u);
    std::vector<std::vector<uint32_t>> outs(n, std::vector<uint32_t>(2 * W));
    std::vector<std::array<uint32_t, 2>> otop(n);
    emu::Wave wave;
    emu::g_wave = &wave;
    auto body = [&](uint32_t ln) {
        emu::t_lane = ln;
        const Big<C> ar;
        for (int i = 0; i < n; ++i) {
            if (ln == 0)
                for (int e = 0; e < 2; ++e) {
                    for (uint32_t k = 0; k < W; ++k) sm[cell_base(W, e) + limb_pos(C, k)] = cases[i].x[e][k];
                    sm[e] = cases[i].top[e];
                }
            emu::sync();
            base_case<C>(ar, sm.data(), LeafOp{cases[i].code | (1u << 18), 0u}, cases[i].s, 2 * N - 1);
            emu::sync();
            if (ln == 0)
                for (int e = 0; e < 2; ++e) {
                    for (uint32_t k = 0; k < W; ++k) outs[i][e * W + k] = sm[cell_base(W, e) + limb_pos(C, k)];
                    otop[i][e] = sm[e];
                }
            emu::sync();
        }
    };
    std::vector<std::thread> th;
    for (uint32_t ln = 0; ln < 64; ++ln) th.emplace_back(body, ln);
    for (auto &t : th) t.join();
    for (int i = 0; i < n; ++i) {
        std::printf("%u %u ", otop[i][0], otop[i][1]);
        for (int e = 0; e < 2; ++e) {
            for (int k = (int)W - 1; k >= 0; --k) std::printf("%08x", outs[i][e * W + k]);
            std::printf(e ? "\n" : " ");
        }
    }
    return 0;
}

int main(int argc, char **argv) {
    if (argc == 3 && std::string(argv[1]) == "records") {
        switch (std::atoi(argv[2])) {
            case 4: return run_records<4>();
            case 8: return run_records<8>();
            case 16: return run_records<16>();
            case 32: return run_records<32>();
            default: return 2;
        }
    }
    if (argc == 3 && std::string(argv[1]) == "plan") {
        switch (std::atoi(argv[2])) {
            case 4: return run_plan<4>();
            case 8: return run_plan<8>();
            case 16: return run_plan<16>();
            case 32: return run_plan<32>();
            default: return 2;
        }
    }
    if (argc < 4) return 2;
    const int C = std::atoi(argv[1]), n = std::atoi(argv[2]);
    const uint64_t seed = std::strtoull(argv[3], nullptr, 0);
    switch (C) {
        case 4: run<4>(n, seed); break;
        case 8: run<8>(n, seed); break;
        case 16: run<16>(n, seed); break;
        case 32: run<32>(n, seed); break;
        default: return 2;
    }
    return 0;
}
