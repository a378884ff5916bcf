// CPU check of the default-shape sweep tables (hq_sweeptab.h): for every
// layer, segment and lane of an N-unit layout with b = 10 low bits, the
// record and the low-pattern row must lead to exactly the states the update
// (12) reads.  A state's position is recomputed independently as the layer
// start plus its colex rank (combinatorial number system):
//   - self + t is the position of m = (T << b) | L;
//   - for a row entry k < q: unit l = slot / 8 is set in L (entries in
//     increasing l) and dn + off / elem is the position of m minus unit l;
//   - for k >= q: unit l = slot / 8 - 16 is clear in L and
//     up + off / elem - C(b, q - 1) is the position of m plus unit l (a
//     wave's staging area holds the down segment, then the up segment);
//   - hi[k] + t is the position of m xor 2^(b + k);
//   - mu_lo and mu_hi are the service-rate sums of the busy units, pmask
//     marks the units with program terms and pstart/pcount the tile's terms.
// Usage: sweeptab_check N   (exit status 0 = pass)
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "hq_sweeptab.h"

static int fails = 0;
#define CHECK(c, ...)                       \
    do {                                    \
        if (!(c)) {                         \
            if (fails++ < 10) {             \
                std::printf(__VA_ARGS__);   \
                std::printf("\n");          \
            }                               \
        }                                   \
    } while (0)

static uint64_t position(uint32_t m, const std::vector<uint32_t>& layer_off) {
    uint64_t r = 0;
    int i = 0;
    const int n = __builtin_popcount(m);
    for (int p = 0; m; ++p, m >>= 1)
        if (m & 1u) r += (uint64_t)hqlayout::binom(p, ++i);
    return layer_off[n] + r;
}

int main(int argc, char** argv) {
    if (argc != 2) return 2;
    const int N = std::atoi(argv[1]), b = HQ_SWEEP_B;
    hqlayout::Layout lay;
    hqlayout::build_layout(N, b, lay);
    const int H = N - b;
    const uint32_t tiles = 1u << H;
    std::vector<double> nu(N);
    for (int u = 0; u < N; ++u) nu[u] = 0.5 + 0.1 * u;
    // a synthetic program layout: tile T has (T * 7 + u) % 3 terms for unit u
    std::vector<uint32_t> prog_off((size_t)tiles * (N + 1));
    uint32_t pos = 0;
    for (uint32_t T = 0; T < tiles; ++T) {
        for (int u = 0; u < N; ++u) {
            prog_off[(size_t)T * (N + 1) + u] = pos;
            pos += (T * 7u + (uint32_t)u) % 3u;
        }
        prog_off[(size_t)T * (N + 1) + N] = pos;
    }
    for (int elem : {8, 4}) {
        const std::vector<LowRow> rows = hqsweeptab::low_rows(lay, nu, elem);
        const std::vector<uint32_t> rec = hqsweeptab::seg_records(lay, prog_off, nu);
        CHECK(rows.size() == (1u << b), "rows %zu", rows.size());
        CHECK(rec.size() == lay.seg_desc.size() * HQ_REC_WORDS, "records %zu", rec.size());
        for (int n = 0; n <= N; ++n) {
            for (uint32_t s = lay.desc_base[n]; s < lay.desc_base[n + 1]; ++s) {
                const uint32_t* w = rec.data() + (size_t)s * HQ_REC_WORDS;
                const uint32_t desc = w[HQ_REC_DESC], T = desc >> 4;
                const int q = (int)(desc & 15u);
                CHECK(desc == lay.seg_desc[s], "desc");
                CHECK(__builtin_popcount(T) + q == n, "class of segment %u in layer %d", s, n);
                double mh = 0.0;
                for (int k = 0; k < H; ++k)
                    if ((T >> k) & 1u) mh += nu[b + k];
                double got;
                std::memcpy(&got, w + HQ_REC_MUHI, sizeof(double));
                CHECK(got == mh, "mu_hi");
                const uint32_t* po = prog_off.data() + (size_t)T * (N + 1);
                CHECK(w[HQ_REC_PSTART] == po[0] && w[HQ_REC_PCOUNT] == po[N] - po[0], "program range");
                for (int u = 0; u < N; ++u)
                    CHECK((((w[HQ_REC_PMASK] >> u) & 1u) != 0) == (po[u + 1] > po[u]), "pmask unit %d", u);
                const uint32_t cnt = (uint32_t)hqlayout::binom(b, q);
                for (uint32_t t = 0; t < cnt; ++t) {
                    const LowRow& r = rows[lay.lo_qstart[q] + t];
                    const uint32_t L = r.L, m = (T << b) | L;
                    CHECK(__builtin_popcount(L) == q, "row class");
                    CHECK(w[HQ_REC_SELF] + t == position(m, lay.layer_off), "self of m=%u", m);
                    double ml = 0.0;
                    int prev = -1;
                    for (int k = 0; k < b; ++k) {
                        const int sl = r.slot[k] / 8;
                        const uint32_t e = r.off[k];
                        CHECK(r.slot[k] % 8 == 0 && e % (uint32_t)elem == 0, "alignment");
                        if (k < q) {
                            const int l = sl;
                            CHECK(l >= 0 && l < b && ((L >> l) & 1u), "down entry %d of L=%u", k, L);
                            CHECK(l > prev, "order");
                            prev = (k == q - 1) ? -1 : l;
                            CHECK(w[HQ_REC_DN] + e / elem == position(m ^ (1u << l), lay.layer_off),
                                  "down neighbour of m=%u unit %d", m, l);
                            CHECK(e / elem < hqlayout::binom(b, q - 1), "down offset in segment");
                            ml += nu[l];
                        } else {
                            const int l = sl - 16;
                            CHECK(l >= 0 && l < b && !((L >> l) & 1u), "up entry %d of L=%u", k, L);
                            CHECK(l > prev, "order");
                            prev = l;
                            const uint32_t dn = q > 0 ? (uint32_t)hqlayout::binom(b, q - 1) : 0u;
                            CHECK(e / elem >= dn, "up offset after the down segment");
                            CHECK(w[HQ_REC_UP] + (e / elem - dn) == position(m | (1u << l), lay.layer_off),
                                  "up neighbour of m=%u unit %d", m, l);
                            CHECK(e / elem - dn < hqlayout::binom(b, q + 1), "up offset in segment");
                            CHECK(e / elem < HQ_SWEEP_STAGE, "staging area");
                        }
                    }
                    CHECK(std::fabs(ml - r.mu_lo) <= 1e-12, "mu_lo");
                    for (int k = 0; k < H; ++k)
                        CHECK(w[HQ_REC_HI + k] + t == position(m ^ (1u << (b + k)), lay.layer_off),
                              "high neighbour of m=%u bit %d", m, b + k);
                }
            }
        }
    }
    if (fails) {
        std::printf("%d failures\n", fails);
        return 1;
    }
    return 0;
}
