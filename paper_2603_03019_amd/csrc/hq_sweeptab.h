// Host tables of the default-shape sweep kernels (hq_sweep.hip): the
// per-segment records and the per-low-pattern rows.  Plain C++ (no HIP
// types), shared by the library and by a CPU checker.
#pragma once

#include <stdint.h>

#include <cstring>
#include <vector>

#include "hq_layout.h"

// Default tile width of the sweep kernels in hq_sweep.hip (b = 10 low bits).
#define HQ_SWEEP_B 10

// Precomputed record of one segment (T, q) of one layer, 32 words, in the
// order the layer's segments are processed (the seg_desc order):
#define HQ_REC_WORDS 32
#define HQ_REC_SELF 0    // start of (T, q) in the state vector
#define HQ_REC_DN 1      // start of (T, q - 1) in layer n - 1 (0 when q = 0)
#define HQ_REC_UP 2      // start of (T, q + 1) in layer n + 1 (0 when q = b)
#define HQ_REC_DESC 3    // (T << 4) | q
#define HQ_REC_PSTART 4  // first program term of tile T
#define HQ_REC_PCOUNT 5  // number of program terms of tile T
#define HQ_REC_PMASK 6   // bit u: unit u has program terms in tile T
#define HQ_REC_MUHI 8    // words 8, 9: sum of nu over the busy high units (FP64)
#define HQ_REC_HI 10     // words 10 + k: start of (T xor 2^k, q) in layer n -+ 1, k < H

// Per low pattern, in the order of lo_unrank (class q, then colex rank t):
// the pattern; for its q set bits (increasing) the byte offset of L minus
// that bit in a wave's staging area, which holds segment (T, q - 1) and
// then segment (T, q + 1); then for its b - q clear bits the byte offset of
// L plus that bit there (one table per element size); the byte offset of
// each entry's weight in a wave's 64-double LDS area (unit l of a set bit:
// l, of a clear bit: 16 + l); and the service-rate sum of the pattern's
// units.
#define HQ_SWEEP_STAGE 424  // staging elements per wave: >= C(10, q - 1) + C(10, q + 1) for every q
struct LowRow {
    uint16_t L;
    uint16_t off[HQ_SWEEP_B];
    uint8_t slot[HQ_SWEEP_B];
    double mu_lo;
};
static_assert(sizeof(LowRow) == 40, "LowRow is read as 40-byte rows");

namespace hqsweeptab {

// Rows of the low patterns in lo_unrank order (class q, then colex rank):
// set bits first (down-neighbour L minus the bit at its rank in class
// q - 1, weight slot l), then clear bits (up-neighbour L plus the bit at
// C(b, q - 1) + its rank in class q + 1, weight slot 16 + l); `elem` is
// the element size the offsets count in.
inline std::vector<LowRow> low_rows(const hqlayout::Layout& lay, const std::vector<double>& nu, int elem) {
    const int b = lay.b;
    const uint32_t lo = 1u << b;
    std::vector<LowRow> rows(lo);
    for (uint32_t i = 0; i < lo; ++i) {
        const uint32_t L = lay.lo_unrank[i];
        LowRow r{};
        r.L = (uint16_t)L;
        int k = 0;
        for (int l = 0; l < b; ++l)
            if ((L >> l) & 1u) {
                r.off[k] = (uint16_t)(lay.lo_rank[L ^ (1u << l)] * (uint32_t)elem);
                r.slot[k++] = (uint8_t)(8 * l);
            }
        for (int l = 0; l < b; ++l)
            if (!((L >> l) & 1u)) {
                const int q = __builtin_popcount(L);
                const uint32_t dn = q > 0 ? (uint32_t)hqlayout::binom(b, q - 1) : 0u;
                r.off[k] = (uint16_t)((dn + lay.lo_rank[L | (1u << l)]) * (uint32_t)elem);
                r.slot[k++] = (uint8_t)(8 * (16 + l));
            }
        double m = 0.0;
        for (int l = 0; l < b; ++l)
            if ((L >> l) & 1u) m += nu[l];
        r.mu_lo = m;
        rows[i] = r;
    }
    return rows;
}

// Records of every layer's segments in seg_desc order (HQ_REC_WORDS words
// each): segment starts of (T, q), (T, q -+ 1) and (T xor 2^k, q), the
// tile's program position and units with terms, and the service-rate sum
// of the tile's busy units.  prog_off: [2^H * (N + 1)] per tile.
inline std::vector<uint32_t> seg_records(const hqlayout::Layout& lay, const std::vector<uint32_t>& prog_off,
                                         const std::vector<double>& nu) {
    const int N = lay.N, b = lay.b, H = lay.H;
    const uint32_t tiles = 1u << H;
    std::vector<uint32_t> rec(lay.seg_desc.size() * (size_t)HQ_REC_WORDS, 0u);
    for (size_t i = 0; i < lay.seg_desc.size(); ++i) {
        const uint32_t desc = lay.seg_desc[i], T = desc >> 4;
        const int q = (int)(desc & 15u);
        uint32_t* w = rec.data() + i * HQ_REC_WORDS;
        w[HQ_REC_SELF] = lay.segoff[(size_t)q * tiles + T];
        w[HQ_REC_DN] = q >= 1 ? lay.segoff[(size_t)(q - 1) * tiles + T] : 0u;
        w[HQ_REC_UP] = q < b ? lay.segoff[(size_t)(q + 1) * tiles + T] : 0u;
        w[HQ_REC_DESC] = desc;
        const uint32_t* po = prog_off.data() + (size_t)T * (N + 1);
        w[HQ_REC_PSTART] = po[0];
        w[HQ_REC_PCOUNT] = po[N] - po[0];
        uint32_t pm = 0;
        for (int u = 0; u < N; ++u)
            if (po[u + 1] > po[u]) pm |= 1u << u;
        w[HQ_REC_PMASK] = pm;
        double mh = 0.0;
        for (int k = 0; k < H; ++k)
            if ((T >> k) & 1u) mh += nu[b + k];
        std::memcpy(w + HQ_REC_MUHI, &mh, sizeof(double));
        for (int k = 0; k < H; ++k) w[HQ_REC_HI + k] = lay.segoff[(size_t)q * tiles + (T ^ (1u << k))];
    }
    return rec;
}

}  // namespace hqsweeptab
