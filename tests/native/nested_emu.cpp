// Host run of the nested Schoenhage-Strassen pointwise product
// (paper_0810_3203_amd/csrc/fermat_nested.hpp, the functions the kernel
// calls), phase by phase in the kernel's order with the lanes taken one after
// another (no phase lets lanes talk to each other between barriers).  It reads
// cases from stdin and prints, per case, the per-limb sums of positive and of
// negative words the kernel hands to its last phase; tests/test_nested_emu.py
// checks that sum_j (pos_j - neg_j) 2^(32 j) = a b mod 2^N+1.
//
// stdin: W, then count, then per case 2W limbs (a, then b) in hex
// stdout: per case 2W numbers in hex (pos_0 .. pos_{W-1}, neg_0 .. neg_{W-1})
//
// With W = 0 it instead runs the inner-cell helpers on constructed cells of
// Z/(2^3072+1) (the N = 65536 configuration): normalize with h far outside
// {0, 1} and at the wrap-around points, and the products involving 2^N'.
// Each output line: the inputs, then the result (limbs in hex, then h).
#include <cstdint>
#include <cstdio>
#include <vector>

#include "fermat_nested.hpp"

// one forward transform of the digit cells, each level's items reading
// before any writes (the kernel's barrier)
template <class NS>
static void forward(int64_t *D) {
    constexpr int K = NS::K, WI = NS::WI, CP = WI + 1;
    constexpr uint32_t HW = K / 2 * WI;
    for (int hs = K / 2; hs >= 1; hs >>= 1) {
        std::vector<int64_t> sv(HW), ev(HW);
        std::vector<uint32_t> xi(HW), yi(HW);
        for (uint32_t e = 0; e < HW; ++e) {
            const uint32_t t = e / WI, d = e - t * WI;
            const uint32_t off = t % hs, o = (t / hs) * 2 * hs + off;
            const int64_t x = D[o * CP + d], y = D[(o + hs) * CP + d];
            uint32_t dd = d + NS::twiddle_limbs((int)off, hs);
            int64_t dv = x - y;
            if (dd >= (uint32_t)WI) {
                dd -= WI;
                dv = -dv;
            }
            sv[e] = x + y;
            ev[e] = dv;
            xi[e] = o * CP + d;
            yi[e] = (o + hs) * CP + dd;
        }
        for (uint32_t e = 0; e < HW; ++e) {
            D[xi[e]] = sv[e];
            D[yi[e]] = ev[e];
        }
    }
}

template <int W>
static void run_case(const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) {
    using NS = tft::nest::Nest<W>;
    constexpr int K = NS::K, WI = NS::WI, WP = NS::WP, NC = NS::NC, G = NS::G, CP = WI + 1, DP = NS::DP;
    constexpr uint32_t KW = K * WI, HW = K / 2 * WI;
    std::vector<uint32_t> sm(NS::WORDS, 0xDEADBEEFu);
    int64_t *D = reinterpret_cast<int64_t *>(sm.data() + NS::D);
    uint32_t *LA = sm.data() + NS::LA, *CWS = sm.data() + NS::CW;
    auto split = [&](const std::vector<uint32_t> &x) {
        constexpr int KPW = NS::PL / G, DPW = (WI + G - 1) / G;
        auto limb = [&](int q) { return x[q]; };
        // every zero write of a cell comes before the piece writes (the
        // kernel's waves do both, on disjoint digits)
        for (int w = 0; w < G; ++w)
            for (int l = 0; l < 64; ++l) {
                const int d0 = w * DPW, d1 = d0 + DPW < WI ? d0 + DPW : WI;
                NS::split_zero(l, d0, d1, D + l * CP);
            }
        for (int w = 0; w < G; ++w)
            for (int l = 0; l < 64; ++l) NS::split_part(limb, l, w * KPW, (w + 1) * KPW, D + l * CP);
    };
    split(a);
    forward<NS>(D);
    for (int l = 0; l < 64; ++l) NS::norm_digits(D + l * CP, LA + l * WP);
    split(b);
    forward<NS>(D);
    for (int l = 0; l < 64; ++l) NS::norm_digits(D + l * CP, sm.data() + NS::D + l * DP);
    auto mac = [](uint64_t (&acc)[NC], uint32_t (&cy)[NC], const uint32_t (&aw)[NC], uint32_t bj) {
        for (int c = 0; c < NC; ++c) {
            const uint64_t p = (uint64_t)aw[c] * bj, s = acc[c] + p;
            cy[c] += s < p ? 1u : 0u;
            acc[c] = s;
        }
    };
    std::vector<uint32_t> outs(G * 64 * NC);
    std::vector<bool> sp(64);
    for (int w = 0; w < G; ++w)
        for (int l = 0; l < 64; ++l) {
            uint32_t out[NC];
            const uint32_t *Bl = sm.data() + NS::D + l * DP;
            sp[l] = NS::geth(LA + l * WP) != 0 || NS::geth(Bl) != 0;
            const int64_t cw = NS::columns(LA + l * WP, Bl, w * NC, out, mac);
            for (int k = 0; k < NC; ++k) outs[(w * 64 + l) * NC + k] = out[k];
            CWS[2 * (w * 64 + l)] = (uint32_t)cw;
            CWS[2 * (w * 64 + l) + 1] = (uint32_t)((uint64_t)cw >> 32);
        }
    for (int w = 0; w < G; ++w)
        for (int l = 0; l < 64; ++l)
            if (!sp[l])
                for (int k = 0; k < NC; ++k) LA[l * WP + w * NC + k] = outs[(w * 64 + l) * NC + k];
    for (int l = 0; l < 64; ++l) {
        uint32_t *Ai = LA + l * WP;
        if (sp[l]) {
            NS::special_product(Ai, sm.data() + NS::D + l * DP, Ai);
        } else {
            int64_t cg[G];
            for (int w = 0; w < G; ++w)
                cg[w] = (int64_t)((uint64_t)CWS[2 * (w * 64 + l) + 1] << 32 | CWS[2 * (w * 64 + l)]);
            NS::settle_columns(Ai, cg);
        }
    }
    for (uint32_t e = 0; e < KW; ++e) {
        const uint32_t i = e / WI, d = e - i * WI;
        int64_t v = LA[i * WP + d];
        if (d == 0) v -= NS::geth(LA + i * WP);
        D[i * CP + d] = v;
    }
    for (int hs = 1; hs <= K / 2; hs <<= 1) {
        std::vector<int64_t> xv(HW), yv(HW);
        std::vector<uint32_t> xi(HW), yi(HW);
        for (uint32_t e = 0; e < HW; ++e) {
            const uint32_t t = e / WI, d = e - t * WI;
            const uint32_t off = t % hs, o = (t / hs) * 2 * hs + off;
            const int64_t x = D[o * CP + d];
            const uint32_t dq = d + NS::twiddle_limbs((int)off, hs);
            const int64_t y = dq < (uint32_t)WI ? D[(o + hs) * CP + dq] : -D[(o + hs) * CP + dq - WI];
            xv[e] = x + y;
            yv[e] = x - y;
            xi[e] = o * CP + d;
            yi[e] = (o + hs) * CP + d;
        }
        for (uint32_t e = 0; e < HW; ++e) {
            D[xi[e]] = xv[e];
            D[yi[e]] = yv[e];
        }
    }
    for (int l = 0; l < 64; ++l) NS::norm_digits(D + l * CP, LA + l * WP);
    for (uint32_t e = 0; e < KW; ++e) {
        const uint32_t i = e / WI, d = e - i * WI;
        D[i * CP + d] = NS::untwist_digit(LA + i * WP, (int)i, (int)d);
    }
    for (int l = 0; l < 64; ++l) {
        NS::norm_digits(D + l * CP, LA + l * WP);
        NS::magnitude(LA + l * WP, LA + l * WP);
    }
    std::vector<uint64_t> pos(W), neg(W);
    for (int j = 0; j < W; ++j) NS::gather(LA, j, pos[j], neg[j]);
    for (int j = 0; j < W; ++j) printf("%llx ", (unsigned long long)pos[j]);
    for (int j = 0; j < W; ++j) printf("%llx ", (unsigned long long)neg[j]);
    printf("\n");
}

static void unit_cases() {
    using NS = tft::nest::Nest<2048>;
    constexpr int WI = NS::WI;
    auto put = [](const uint32_t *c) {
        for (int m = 0; m < WI; ++m) printf("%x ", c[m]);
        printf("%d", NS::geth(c));
    };
    auto fill = [](uint32_t *c, uint32_t v, int32_t h) {
        for (int m = 0; m < WI; ++m) c[m] = v;
        NS::seth(c, h);
    };
    uint32_t c[NS::WP], d[NS::WP];
    const uint32_t vals[] = {0u, 0xFFFFFFFFu, 5u, 0x80000000u};
    const int64_t hs[] = {0, 1, -1, 2, -2, (int64_t)1 << 40, -((int64_t)1 << 40), 12345, -77};
    for (uint32_t v : vals)
        for (int64_t h : hs) {
            fill(c, v, 0);
            if (v == 5u) c[WI - 1] = 0x1234u;  // a value that is not a single repeated word
            printf("N ");
            put(c);
            printf(" %lld ", (long long)h);
            NS::normalize(c, h);
            put(c);
            printf("\n");
        }
    // products with 2^N' (h = 1, limbs 0) on either side
    const uint32_t others[] = {0u, 1u, 0xFFFFFFFFu, 0x9E3779B9u};
    for (int side = 0; side < 3; ++side)
        for (uint32_t v : others) {
            fill(c, 0u, 1);
            fill(d, v, 0);
            if (v == 1u)
                for (int m = 1; m < WI; ++m) d[m] = 0u;
            const uint32_t *x = side == 1 ? d : c, *y = side == 1 ? c : d;
            if (side == 2) y = c;  // 2^N' times 2^N'
            printf("S ");
            put(x);
            printf(" ");
            put(y);
            printf(" ");
            uint32_t out[NS::WP];
            NS::special_product(x, y, out);
            put(out);
            printf("\n");
        }
}

int main() {
    int W, count;
    if (scanf("%d", &W) != 1) return 2;
    if (W == 0) {
        unit_cases();
        return 0;
    }
    if (scanf("%d", &count) != 1) return 2;
    for (int c = 0; c < count; ++c) {
        std::vector<uint32_t> a(W), b(W);
        for (int q = 0; q < W; ++q)
            if (scanf("%x", &a[q]) != 1) return 2;
        for (int q = 0; q < W; ++q)
            if (scanf("%x", &b[q]) != 1) return 2;
        if (W == 512)
            run_case<512>(a, b);
        else if (W == 1024)
            run_case<1024>(a, b);
        else if (W == 2048)
            run_case<2048>(a, b);
        else if (W == 4096)
            run_case<4096>(a, b);
        else
            return 3;
    }
    return 0;
}
