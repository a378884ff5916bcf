// CPU check of the layer kernels' index arithmetic (hq_layout.h): for every
// layer, segment and lane, the position is a bijection onto [0, 2^N) equal
// to layer start + colex rank, every neighbour index the kernels form is in
// bounds and points at m xor 2^u, and every segment-table read is in bounds.
// Usage: layout_check N b   (exit status 0 = pass)
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hq_layout.h"

using namespace hqlayout;

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

// bounds-checked view of a table, used as the kernels' pointer type
template <typename T>
struct Checked {
    const std::vector<T>* v;
    T operator[](uint64_t i) const {
        CHECK(i < v->size(), "table read %llu out of %zu", (unsigned long long)i, v->size());
        return i < v->size() ? (*v)[i] : T(0);
    }
};

static uint32_t colex_rank(uint32_t m) {
    uint32_t r = 0;
    int i = 0;
    for (int p = 0; m; ++p, m >>= 1)
        if (m & 1u) r += (uint32_t)binom(p, ++i);
    return r;
}

int main(int argc, char** argv) {
    const int N = std::atoi(argv[1]), b = std::atoi(argv[2]);
    Layout Lo;
    build_layout(N, b, Lo);
    const int H = N - b;
    const uint32_t tiles = 1u << H, S = 1u << N;
    Checked<uint32_t> segoff{&Lo.segoff};
    Checked<uint16_t> rank{&Lo.lo_rank};
    std::vector<int64_t> pos_of(S, -1);
    std::vector<char> taken(S, 0);
    for (int n = 0; n <= N; ++n) {
        for (uint32_t g = Lo.desc_base[n]; g < Lo.desc_base[n + 1]; ++g) {
            const uint32_t d = Lo.seg_desc[g];
            const int q = (int)(d & 15u);
            const uint32_t Tb = d >> 4;
            CHECK(q <= b && Tb < tiles && __builtin_popcount(Tb) + q == n, "bad descriptor");
            const uint32_t self = segoff[seg_index(q, Tb, tiles)];
            const uint32_t cnt = (uint32_t)binom(b, q);
            CHECK(self >= Lo.layer_off[n] && self + cnt <= Lo.layer_off[n + 1], "segment outside its layer");
            for (uint32_t t = 0; t < cnt; ++t) {
                const uint32_t L = Lo.lo_unrank[Lo.lo_qstart[q] + t];
                const uint32_t m = (Tb << b) | L;
                const uint32_t pos = self + t;
                CHECK(pos < S && !taken[pos], "position %u reused or out of range", pos);
                CHECK(pos == Lo.layer_off[n] + colex_rank(m), "position is not the colex rank");
                if (pos < S) taken[pos] = 1;
                pos_of[m] = pos;
            }
        }
    }
    for (uint32_t p = 0; p < S; ++p) CHECK(taken[p], "position %u never filled", p);
    for (uint32_t m = 0; m < S; ++m) {
        const int n = __builtin_popcount(m);
        const uint32_t Tb = m >> b, L = m & ((1u << b) - 1u);
        const int q = __builtin_popcount(L);
        const uint32_t self = segoff[seg_index(q, Tb, tiles)];
        const uint32_t t = (uint32_t)pos_of[m] - self;
        for (int k = 0; k < H; ++k) {
            const uint32_t nb = m ^ (1u << (b + k));
            const bool exists = (Tb >> k) & 1u ? n >= 1 : n < N;
            if (!exists) continue;
            const uint32_t idx = high_neighbour(segoff, tiles, q, Tb, k, t);
            CHECK(idx < S && idx == pos_of[nb], "high neighbour N=%d b=%d m=%u k=%d", N, b, m, k);
        }
        const uint32_t offDlo = low_down_segment(segoff, tiles, q, Tb);
        const uint32_t offUlo = low_up_segment(segoff, tiles, q, b, Tb);
        for (int l = 0; l < b; ++l) {
            const uint32_t idx = low_neighbour(L, l, offDlo, offUlo, rank);
            CHECK(idx < S && idx == pos_of[m ^ (1u << l)], "low neighbour N=%d b=%d m=%u l=%d", N, b, m, l);
        }
    }
    if (fails) std::printf("N=%d b=%d: %d failures\n", N, b, fails);
    return fails ? 1 : 0;
}
