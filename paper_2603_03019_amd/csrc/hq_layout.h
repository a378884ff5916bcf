// State-vector layout of the layer sweep, shared by the host table builders,
// the HIP kernels and the CPU layout checker (plain C++, no HIP types).
//
// Layer n holds the C(N, n) states with n busy units in colexicographic
// order (increasing bitmask).  A state m = (T << b) | L splits into a high
// tile T (bits b..N-1) and a low pattern L (bits 0..b-1, q = |L| set).  The
// states of one (T, q) form a contiguous segment of C(b, q) entries in colex
// order of L.  The segment's position is
//     layer_off[|T| + q] + sum_i C(b + k_i, q + i)
// over the set bits k_1 < k_2 < ... of T (i = 1, 2, ...): the colex rank of
// the high part.  Flipping a high bit keeps L, hence the lane offset t.
#pragma once

#include <stdint.h>

#include <vector>

#ifdef __HIPCC__
#define HQ_HD __host__ __device__ __forceinline__
#else
#define HQ_HD inline
#endif

namespace hqlayout {

inline double binom(int n, int k) {
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return (double)(long long)(r + 0.5);
}

// Index of the segment table entry of (T, q).
HQ_HD uint64_t seg_index(int q, uint32_t Tb, uint32_t tiles) { return (uint64_t)q * tiles + Tb; }

// Position of the high-bit neighbour (T xor 2^k, q) at lane t.
template <typename Ptr>
HQ_HD uint32_t high_neighbour(Ptr segoff, uint32_t tiles, int q, uint32_t Tb, int k, uint32_t t) {
    return segoff[seg_index(q, Tb ^ (1u << k), tiles)] + t;
}

// Start of the low-bit neighbour segments (T, q - 1) and (T, q + 1); 0 when absent.
template <typename Ptr>
HQ_HD uint32_t low_down_segment(Ptr segoff, uint32_t tiles, int q, uint32_t Tb) {
    return q >= 1 ? segoff[seg_index(q - 1, Tb, tiles)] : 0u;
}
template <typename Ptr>
HQ_HD uint32_t low_up_segment(Ptr segoff, uint32_t tiles, int q, int b, uint32_t Tb) {
    return q < b ? segoff[seg_index(q + 1, Tb, tiles)] : 0u;
}

// Position of the low-bit neighbour m xor 2^l (l < b) given the two segment starts.
template <typename RankPtr>
HQ_HD uint32_t low_neighbour(uint32_t L, int l, uint32_t offDlo, uint32_t offUlo, RankPtr rank) {
    const uint32_t bit = 1u << l;
    return ((L & bit) ? offDlo : offUlo) + rank[L ^ bit];
}

// ---------------------------------------------------------------- host side

struct Layout {
    int N = 0, b = 0, H = 0;
    std::vector<uint32_t> layer_off;  // [N + 2]
    std::vector<uint16_t> lo_unrank;  // [2^b] low patterns by (popcount, value)
    std::vector<uint16_t> lo_rank;    // [2^b] colex rank inside the popcount class
    std::vector<uint32_t> lo_qstart;  // [b + 2]
    std::vector<uint32_t> segoff;     // [(b + 1) * 2^H]
    std::vector<uint32_t> seg_desc;   // per layer: (T << 4) | q in memory order
    std::vector<uint32_t> desc_base;  // [N + 2]
};

inline void build_layout(int N, int b, Layout& Lo) {
    Lo.N = N;
    Lo.b = b;
    Lo.H = N - b;
    const int H = Lo.H;
    Lo.layer_off.assign(N + 2, 0);
    for (int n = 0; n <= N; ++n) Lo.layer_off[n + 1] = Lo.layer_off[n] + (uint32_t)binom(N, n);
    const uint32_t lo = 1u << b;
    Lo.lo_unrank.clear();
    Lo.lo_rank.assign(lo, 0);
    Lo.lo_qstart.assign(b + 2, 0);
    for (int q = 0; q <= b; ++q) {
        Lo.lo_qstart[q] = (uint32_t)Lo.lo_unrank.size();
        uint32_t r = 0;
        for (uint32_t L = 0; L < lo; ++L)
            if (__builtin_popcount(L) == q) {
                Lo.lo_unrank.push_back((uint16_t)L);
                Lo.lo_rank[L] = (uint16_t)r++;
            }
    }
    Lo.lo_qstart[b + 1] = lo;
    const uint32_t tiles = 1u << H;
    Lo.segoff.assign((size_t)(b + 1) * tiles, 0);
    for (uint32_t T = 0; T < tiles; ++T) {
        const int h = __builtin_popcount(T);
        for (int q = 0; q <= b; ++q) {
            uint32_t off = 0;
            int i = 0;
            for (int k = 0; k < H; ++k)
                if ((T >> k) & 1u) off += (uint32_t)binom(b + k, q + (++i));
            Lo.segoff[seg_index(q, T, tiles)] = Lo.layer_off[h + q] + off;
        }
    }
    Lo.seg_desc.clear();
    Lo.desc_base.assign(N + 2, 0);
    for (int n = 0; n <= N; ++n) {
        Lo.desc_base[n] = (uint32_t)Lo.seg_desc.size();
        // processing order = memory order (tile T ascending); each XCD takes
        // one contiguous eighth of it
        for (uint32_t T = 0; T < tiles; ++T) {
            const int q = n - __builtin_popcount(T);
            if (q >= 0 && q <= b) Lo.seg_desc.push_back((T << 4) | (uint32_t)q);
        }
    }
    Lo.desc_base[N + 1] = (uint32_t)Lo.seg_desc.size();
}

}  // namespace hqlayout
