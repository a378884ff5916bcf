// CPU check of the per-tile dispatch tables (hq_tables.h): for sampled
// states, every busy unit's arrival coefficient rebuilt from the tables the
// sweep reads (tile-uniform part + program terms whose low mask lies in the
// state's low bits, in relabelled units) must equal the coefficient of
// Algorithm 3 given in the input (from the oracle).
// Usage: tables_check FILE   (exit status 0 = pass)
// FILE (little-endian): int32 N, J, b, K; double lam[J]; double nu[N];
// int32 pref[J*N]; uint32 states[K] (caller's unit labels);
// double expect[K*N] (a(m, u) for the caller's unit u; 0 when u is idle).
#include <cmath>
#include <cstdio>
#include <vector>

#include "hq_tables.h"

template <typename T>
static bool rd(FILE* f, T* p, size_t n) {
    return std::fread(p, sizeof(T), n, f) == n;
}

int main(int argc, char** argv) {
    if (argc != 2) return 2;
    FILE* f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t hdr[4];
    if (!rd(f, hdr, 4)) return 2;
    const int N = hdr[0], J = hdr[1], b = hdr[2], K = hdr[3];
    std::vector<double> lam(J), nu(N), expect((size_t)K * N);
    std::vector<int32_t> pref((size_t)J * N);
    std::vector<uint32_t> states(K);
    if (!rd(f, lam.data(), J) || !rd(f, nu.data(), N) || !rd(f, pref.data(), pref.size()) ||
        !rd(f, states.data(), K) || !rd(f, expect.data(), expect.size()))
        return 2;
    std::fclose(f);

    const std::vector<int> orig = hqtables::relabel(N, J, lam.data(), nu.data(), pref.data());
    std::vector<int> newlab(N);
    for (int u = 0; u < N; ++u) newlab[orig[u]] = u;
    std::vector<int32_t> rp(pref.size());
    for (size_t i = 0; i < rp.size(); ++i) rp[i] = newlab[pref[i]];
    std::vector<double> tcoef;
    std::vector<uint32_t> prog_off;
    std::vector<ProgTerm> prog;
    hqtables::build_programs(N, b, hqtables::build_terms(N, J, lam.data(), rp), tcoef, prog_off, prog);

    const uint32_t lomask = (1u << b) - 1u;
    const size_t tiles = (size_t)1 << (N - b);
    int bad = 0;
    double worst = 0.0;
    for (int k = 0; k < K; ++k) {
        const uint32_t m = states[k];
        uint32_t mr = 0;
        for (int u = 0; u < N; ++u)
            if ((m >> u) & 1u) mr |= 1u << newlab[u];
        const size_t T = mr >> b;
        const uint32_t L = mr & lomask;
        if (T >= tiles || tcoef.size() != tiles * N || prog_off.size() != tiles * (N + 1)) {
            std::printf("table sizes\n");
            return 1;
        }
        for (int u = 0; u < N; ++u) {
            if (!((m >> u) & 1u)) continue;
            const int ur = newlab[u];
            double c = tcoef.at(T * N + ur);
            const uint32_t i0 = prog_off.at(T * (N + 1) + ur), i1 = prog_off.at(T * (N + 1) + ur + 1);
            if (i0 > i1 || i1 > prog.size()) {
                std::printf("program range\n");
                return 1;
            }
            for (uint32_t i = i0; i < i1; ++i) {
                const ProgTerm& t = prog.at(i);
                if (t.mask & ~lomask) {
                    std::printf("mask outside the low bits\n");
                    return 1;
                }
                if ((L & t.mask) == t.mask) c += t.rate;
            }
            const double want = expect[(size_t)k * N + u];
            const double err = std::fabs(c - want) / std::fmax(std::fabs(want), 1e-300);
            if (want == 0.0 ? c != 0.0 : err > 1e-13) {
                if (bad++ < 10) std::printf("state %u unit %d: tables %.17g, Algorithm 3 %.17g\n", m, u, c, want);
            }
            if (want != 0.0 && err > worst) worst = err;
        }
    }
    std::printf("N=%d b=%d states=%d terms=%zu max relative error %.3g\n", N, b, K, prog.size(), worst);
    return bad ? 1 : 0;
}
